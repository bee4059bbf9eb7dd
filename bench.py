"""Benchmark: Hybrid LSLU iterations per second on one MI355X.

A step is one full Hybrid LSLU solve of the workload (every iteration of the
basis recurrence, the projected problems with weighted-GCV lambda for every k,
all iterates x_k and the copy of the small results to the host), with the
operator and b already resident in HBM.  ``value`` is iterations per second
(maxiter * steps / elapsed).

Default workload ``tomo128``: 128x128 parallel-beam tomography, 180 angles x 181
bins (m = 32580, n = 16384, CSR with bilinear ray-length weights), 2% noise,
100 iterations, FP32 (the mixed-precision mode: FP32 operator/bases/vectors,
FP64 sums, projected problem and pivot divisions).  The FP64 plain mode is
timed on the same problem and both relative errors are reported.

The JSON line also carries the roofline of the dominant kernel -- the
half-iteration kernel of the recurrence (one launch per half-iteration), timed
by the library with HIP events on the stream it launches on -- and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("recurrence.hip", "device_common.hpp", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_2409_05239_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _load_traffic(kernel, workload, prec):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    absent, taken in another precision mode or on a different kernel source."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"{workload}:{prec}:{kernel}")
    if not ent or ent.get("source_hash") != _kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def csr_spmv_bytes(nnz, rows, cols, vsz, esz):
    """Algorithmic bytes of one CSR product: values + column indices, row
    pointers, the input vector once and the output once."""
    return nnz * (vsz + 4) + 4 * (rows + 1) + esz * cols + esz * rows


def recurrence_bytes(prob, K, vsz, esz):
    """Algorithmic HBM bytes of the 2K + 1 launches of the recurrence: per
    half-iteration the operator product (CSR: values, indices, row pointers,
    input once, output once), the earlier basis vectors of the side once, the
    pivot mask, and the previous vector read and written once normalised; the
    last launch only normalises d_{K+1}."""
    m, n = prob.m, prob.n
    if prob.kind == "csr":
        op = {1: csr_spmv_bytes(prob.nnz, n, m, vsz, esz),   # A^T: n rows
              0: csr_spmv_bytes(prob.nnz, m, n, vsz, esz)}   # A:   m rows
    else:
        op = {1: esz * (m + n), 0: esz * (m + n)}
    total = 0
    for k in range(1, K + 1):
        total += op[1] + esz * n * (k - 1) + n + 2 * esz * m   # l side
        total += op[0] + esz * m * k + m + 2 * esz * n         # d side
    total += 2 * esz * m
    return total


def run(args):
    import numpy as np
    import torch

    from paper_2409_05239_amd import capi
    from workloads import CONFIGS, lambda_grid

    cfg = CONFIGS[args.workload]
    prob = cfg["make"]()
    K = args.iters or cfg["iters"]
    prec = args.precision or cfg["precision"]
    grid = lambda_grid()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # The library launches on this stream; every event below is recorded on it.
    stream = torch.cuda.Stream(device=dev)
    ctx = capi.lslu_create(0, stream=stream)

    def setup(p):
        dt = torch.float64 if p == "fp64" else torch.float32
        op = capi.make_operator(ctx, prob, capi.PRECISIONS[p])
        b = torch.tensor(prob.b, dtype=dt, device=dev)
        X = torch.zeros((K, prob.n), dtype=dt, device=dev)
        x = torch.zeros(prob.n, dtype=dt, device=dev)
        torch.cuda.synchronize()
        return op, b, X, x

    sample = None
    if args.pivot_sample > 0:  # the sampled-pivot variant (Section 2.2)
        from workloads import pivot_sample_lists
        sample = (pivot_sample_lists(prob.m, prob.n, K, args.pivot_sample, seed=0),
                  args.pivot_sample)

    def solve(op, b, X, x, timing=False):
        return capi.lslu_solve(ctx, op, b, K, reg=cfg["reg"], lam=cfg.get("lam", 0.0), grid=grid,
                               grid_relative=cfg["grid_relative"], X=X, x_out=x,
                               timing=timing, pivot_sample=sample)

    def timed(p, steps, warmup):
        op, b, X, x = setup(p)
        for _ in range(warmup):
            solve(op, b, X, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st, _, info = solve(op, b, X, x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Xh = X.double().cpu().numpy()
        xt = prob.x_true
        errs = np.linalg.norm(Xh[:info["k_done"]] - xt[None, :], axis=1) / np.linalg.norm(xt)
        # one more solve with the library's phase events (eager launches)
        _, _, tinfo = solve(op, b, X, x, timing=True)
        torch.cuda.synchronize()
        return op, el, info, errs, tinfo["timing"]

    print(f"[bench] workload={args.workload} m={prob.m} n={prob.n} nnz={prob.nnz} "
          f"K={K} prec={prec}", flush=True)
    if args.calibrate_copy:
        # A plain device copy of known size (256 MiB read + 256 MiB written),
        # used to scale the FETCH_SIZE / WRITE_SIZE counters.
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    op, el, info, errs, tm = timed(prec, args.steps, args.warmup)
    ms = el / args.steps * 1e3
    print(f"[bench] {prec}: {ms:.3f} ms/step", flush=True)
    fp64 = None
    if prec != "fp64" and not args.no_fp64:
        op64, el64, info64, errs64, _ = timed("fp64", args.steps, args.warmup)
        fp64 = dict(iters_per_s=K * args.steps / el64, ms_per_step=el64 / args.steps * 1e3,
                    rel_err_final=float(errs64[-1]), rel_err_min=float(errs64.min()),
                    k_min=int(errs64.argmin()) + 1)
        capi.lslu_op_destroy(op64)
        print(f"[bench] fp64: {fp64['ms_per_step']:.3f} ms/step", flush=True)

    # Dominant kernel: the half-iteration kernel of the recurrence.  Its
    # average launch duration is the recurrence's device time (HIP events the
    # library records on its stream around the 2K + 1 launches) per launch.
    esz = 8 if prec == "fp64" else 4
    vsz = {"fp64": 8, "fp32": 4, "bf16op": 2, "fp16op": 2, "fp8op": 1}[prec]
    n_launch = tm["n_recurrence_launches"]
    t_launch = tm["t_recurrence_ms"] * 1e-3 / n_launch
    nbytes = recurrence_bytes(prob, K, vsz, esz) / n_launch
    kname = "k_half_rows" if prob.kind in ("csr", "dense") else "k_half_psf"
    achieved = nbytes / t_launch / 1e9
    roof = dict(bound="hbm", kernel=f"{kname} (one half-iteration: product, "
                "elimination, pivot)", achieved=round(achieved, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=_load_traffic(kname, args.workload, prec),
                us_per_launch=round(t_launch * 1e6, 3), bytes_per_launch=int(nbytes),
                launches_per_step=n_launch,
                phase_ms=dict(recurrence=round(tm["t_recurrence_ms"], 4),
                              projected=round(tm["t_projected_ms"], 4),
                              assemble=round(tm["t_assemble_ms"], 4)))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, cfg, grid, args.cpu_iters or K)
    capi.lslu_op_destroy(op)
    capi.lslu_destroy(ctx)

    out = {
        "metric": "Hybrid LSLU iters/s + % HBM roofline, mixed vs FP64 plain at equal rel. error",
        "value": round(K * args.steps / el, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16op": "bf16-op/f32", "fp16op": "f16-op/f32",
                  "fp8op": "f8-op/f32"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "m": prob.m, "n": prob.n,
                   "nnz": prob.nnz, "iters": K, "precision": prec,
                   "reg": cfg["reg"], "grid_relative": cfg["grid_relative"],
                   "pivot_sample": args.pivot_sample or None},
        "rel_err_final": float(errs[-1]),
        "rel_err_min": float(errs.min()),
        "k_min": int(errs.argmin()) + 1,
        "k_stop": int(info["k_stop"]),
        "status": int(info["status"]),
        "fp64_plain": fp64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(prob, cfg, grid, iters):
    """The FP64 oracle (as is) on the first ``iters`` iterations of the same
    workload, single-threaded BLAS; iterations per second."""
    from threadpoolctl import threadpool_limits

    from oracle import RegParam, make_operator
    from oracle.hessenberg import hybrid_lslu

    op = make_operator(prob)
    reg = RegParam(cfg["reg"], grid=grid, grid_relative=cfg["grid_relative"])
    times = []
    with threadpool_limits(limits=1):
        for _ in range(3):
            t0 = time.perf_counter()
            hybrid_lslu(op, prob.b, iters, reg)
            times.append(time.perf_counter() - t0)
    el = sorted(times)[1]
    return {"value": round(iters / el, 3), "unit": "iters/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} of {cfg['iters']} iterations of the same workload, "
                      f"median of 3 runs of {el:.2f} s (FP64 NumPy/SciPy, one thread)"}


def vjp_bytes(m, n, K, esz):
    """Algorithmic HBM bytes of one reverse pass (lslu_vjp at k = K) with
    every basis vector formed: each array the pass needs is read (or written)
    once per kernel that needs it.  Per iteration kk (K down to 1):
    d-side: dots of dbar_{kk+1} (+ the l-side product) with d_1..d_{kk+1},
    the update that writes the product input and updates dbar_1..dbar_kk
    (read and write), and the product with A^T; l-side: the same with n, kk
    columns, kk-1 updated columns and the product with A.  Start: the dots
    and update of d_1.  Set-up: clearing Dbar, Lbar = xbar y^T and
    ybar = L^T xbar."""
    tot = (K + 1) * m + (K + 1) * n + (K + 1) * n
    for kk in range(K, 0, -1):
        v2 = 1 if kk < K else 0
        tot += (kk + 1) * m + (1 + v2) * m               # d-side dots
        tot += (1 + v2) * m + m + 2 * kk * m             # d-side update
        tot += m + n                                     # A^T product
        tot += kk * n + 2 * n                            # l-side dots
        tot += 2 * n + n + 2 * (kk - 1) * n              # l-side update
        tot += n + m                                     # A product
    tot += m + 2 * m + 2 * m + m                         # start
    return tot * esz


def run_vjp(args):
    """Forward solve + reverse pass (lslu_vjp) of the differentiable workload:
    512 x 512 deblurring, 15 x 15 PSF, 40 iterations, fixed lambda = 0.01,
    loss ||x_K - x_true||^2.  value = iterations per second of forward plus
    reverse; the forward and reverse times are also reported apart."""
    import numpy as np
    import torch

    from paper_2409_05239_amd import capi
    from workloads import CONFIGS

    cfg = CONFIGS["deblur512"]
    prob = cfg["make"]()
    K, lam = cfg["iters"], cfg["lam"]
    prec = args.precision or cfg["precision"]
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    ctx = capi.lslu_create(0, stream=stream)
    op = capi.make_operator(ctx, prob, capi.PRECISIONS[prec])
    with torch.cuda.stream(stream):
        b = torch.tensor(prob.b, dtype=dt, device=dev)
        xt = torch.tensor(prob.x_true, dtype=dt, device=dev)
        x = torch.zeros(prob.n, dtype=dt, device=dev)
        xbar = torch.zeros(prob.n, dtype=dt, device=dev)
        bbar = torch.zeros(prob.m, dtype=dt, device=dev)
    torch.cuda.synchronize()

    def forward():
        st, _, info = capi.lslu_solve(ctx, op, b, K, reg="fixed", lam=lam, x_out=x)
        with torch.cuda.stream(stream):
            torch.sub(x, xt, out=xbar)
            xbar.mul_(2.0)
        return info

    def reverse(k):
        return capi.lslu_vjp(ctx, op, k, xbar, bbar)

    for _ in range(args.warmup):
        info = forward()
        reverse(info["k_done"])
    torch.cuda.synchronize()
    t_f = t_r = 0.0
    for _ in range(args.steps):
        t0 = time.perf_counter()
        info = forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, lam_bar = reverse(info["k_done"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_f += t1 - t0
        t_r += t2 - t1
    t_f /= args.steps
    t_r /= args.steps
    k = info["k_done"]
    esz = 8 if prec == "fp64" else 4
    rb = vjp_bytes(prob.m, prob.n, k, esz)
    loss = float(((x - xt) ** 2).sum())
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import make_operator
        from oracle.gradient import vjp_directional
        oop = make_operator(prob)
        pt = list(info["piv_t"][:k + 1])
        pg = list(info["piv_g"][:k])
        xb = xbar.double().cpu().numpy()
        v = np.random.default_rng(0).standard_normal(prob.m)
        c0 = time.perf_counter()
        vjp_directional(oop, prob.b, k, lam, pt, pg, xb, v)
        el = time.perf_counter() - c0
        cpu = {"value": round(1.0 / el, 4), "unit": "directional derivatives/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one complex-step directional derivative of the same loss "
                         f"({el:.1f} s, FP64 NumPy/SciPy); the whole gradient needs "
                         f"m = {prob.m} of them"}
    capi.lslu_op_destroy(op)
    capi.lslu_destroy(ctx)
    out = {
        "metric": "Differentiable Hybrid LSLU: forward + reverse iterations/s",
        "value": round(k / (t_f + t_r), 1),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t_f + t_r) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "deblur512: 512x512 image, 15x15 Gaussian PSF (sigma 2), "
                               "40 iterations, fixed lambda 0.01, loss ||x_K - x_true||^2",
                   "precision": prec},
        "forward_ms": round(t_f * 1e3, 4),
        "reverse_ms": round(t_r * 1e3, 4),
        "reverse_roofline": {"bound": "hbm", "achieved": round(rb / t_r / 1e9, 1),
                             "peak": 8000.0, "unit": "GB/s",
                             "frac": round(rb / t_r / 1e9 / 8000.0, 4),
                             "bytes": rb, "traffic": None},
        "loss": loss,
        "lambda_bar": lam_bar,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Many uneven problems (workloads.batch_problems: tomography and deblurring
    of different sizes), BF16 operator with FP32 bases, 60 iterations each.
    value: all problems as asynchronous solves on S contexts (one stream
    each), in waves of S.  Also timed: the same one at a time, FP64 one at a
    time, and for the tomography (CSR) half alone the merged batch
    (lslu_solve_batch: each recurrence launch covers every problem) against
    waves on S contexts and one at a time.  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2409_05239_amd import capi
    from workloads import batch_problems, lambda_grid

    P, S, K = args.batch, args.contexts, 60
    probs = batch_problems(P, seed=0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    grid = lambda_grid()
    rr = [capi.lslu_create(0) for _ in range(S)]  # round-robin contexts

    def prepare(prec, ctxs, sel):
        dt = torch.float64 if prec == "fp64" else torch.float32
        items = []
        for i, prob in enumerate(sel):
            c = ctxs[i % len(ctxs)]
            op = capi.make_operator(c, prob, capi.PRECISIONS[prec])
            items.append((c, op, torch.tensor(prob.b, dtype=dt, device=dev),
                          torch.zeros((K, prob.n), dtype=dt, device=dev)))
        torch.cuda.synchronize()
        return items

    def release(items):
        for it in items:
            capi.lslu_op_destroy(it[1])

    def solve(it, asynchronous=False):
        c, op, b, X = it
        return capi.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True,
                               X=X, asynchronous=asynchronous)

    def one_at_a_time(items):
        for it in items:
            solve(it)

    def concurrent(items):
        for w in range(0, len(items), S):
            wave = items[w:w + S]
            pend = [solve(it, asynchronous=True) for it in wave]
            for it, pd in zip(wave, pend):
                capi.lslu_wait(it[0], pd)

    def merged(items):
        capi.lslu_solve_batch([it[0] for it in items], [it[1] for it in items],
                              [it[2] for it in items], K, reg="wgcv", grid=grid,
                              grid_relative=True)

    def merged_groups(groups):
        # problems of similar size merged, the groups side by side (one host
        # thread each; the library call releases the interpreter)
        import threading
        ths = [threading.Thread(target=merged, args=(g,)) for g in groups]
        for t in ths:
            t.start()
        for t in ths:
            t.join()

    def timed(fn, items):
        for _ in range(args.warmup):
            fn(items)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn(items)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    def errors(items, sel):
        errs = []
        for it, prob in zip(items, sel):
            X = it[3].double().cpu().numpy()
            e = np.linalg.norm(X - prob.x_true[None, :], axis=1) / np.linalg.norm(prob.x_true)
            errs.append(float(e.min()))
        return errs

    lo = prepare("bf16op", rr, probs)
    t_conc = timed(concurrent, lo)
    t_seq = timed(one_at_a_time, lo)
    errs = errors(lo, probs)
    release(lo)
    hi = prepare("fp64", rr, probs)
    t_64 = timed(one_at_a_time, hi)
    errs64 = errors(hi, probs)
    release(hi)
    tomo = [p for p in probs if p.kind == "csr"]
    own = [capi.lslu_create(0) for _ in tomo]  # the merged batch: one context each
    mo = prepare("bf16op", own, tomo)
    t_tm = timed(merged, mo)
    order = sorted(range(len(tomo)), key=lambda i: tomo[i].m)
    ng = 4
    groups = [[mo[i] for i in order[g::ng]] for g in range(ng)]  # interleaved by size
    groups = [[mo[i] for i in order[g * len(order) // ng:(g + 1) * len(order) // ng]]
              for g in range(ng)]  # contiguous size classes
    t_tg = timed(merged_groups, groups)
    release(mo)
    for c in own:
        capi.lslu_destroy(c)
    to = prepare("bf16op", rr, tomo)
    t_tc = timed(concurrent, to)
    t_ts = timed(one_at_a_time, to)
    release(to)
    for c in rr:
        capi.lslu_destroy(c)
    it_total = P * K
    it_tomo = len(tomo) * K
    out = {
        "metric": "Batched Hybrid LSLU problem-iterations/s (uneven problems, concurrent contexts)",
        "value": round(it_total / t_conc, 1),
        "unit": "problem-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_conc * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-op/f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {P} uneven problems (tomography 32-96, deblur 64-256)",
                   "iters": K, "contexts": S, "reg": "wgcv", "grid_relative": True},
        "one_at_a_time": {"value": round(it_total / t_seq, 1), "ms_per_step": round(t_seq * 1e3, 3)},
        "fp64_one_at_a_time": {"value": round(it_total / t_64, 1), "ms_per_step": round(t_64 * 1e3, 3)},
        "tomography_half": {"problems": len(tomo),
                            "merged_launches": round(it_tomo / t_tm, 1),
                            "merged_by_size_4_threads": round(it_tomo / t_tg, 1),
                            "concurrent": round(it_tomo / t_tc, 1),
                            "one_at_a_time": round(it_tomo / t_ts, 1)},
        "median_min_rel_err": {"bf16op": float(np.median(errs)), "fp64": float(np.median(errs64))},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tomo128")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--cpu-iters", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--batch", type=int, default=0,
                    help="batched mode: number of uneven problems (0: the default workload)")
    ap.add_argument("--contexts", type=int, default=8,
                    help="batched mode: contexts (streams) solving concurrently")
    ap.add_argument("--pivot-sample", type=int, default=0,
                    help="sampled pivots: sample size per search (0: full searches)")
    ap.add_argument("--vjp", action="store_true",
                    help="time forward + reverse pass of the differentiable "
                         "deblurring workload (512x512, 15x15 PSF, 40 iterations)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the "
              "library has no multi-GPU path (how it would shard is described "
              "with the design)", file=sys.stderr)
        sys.exit(2)
    if args.vjp:
        run_vjp(args)
    elif args.batch > 0:
        run_batch(args)
    else:
        run(args)


if __name__ == "__main__":
    main()
