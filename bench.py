"""Benchmark: Hybrid LSLU iterations per second on one MI355X.

A step is one full Hybrid LSLU solve of the workload (every iteration of the
basis recurrence, the projected problems with weighted-GCV lambda for every k,
all iterates x_k and the copy of the small results to the host), with the
operator and b already resident in HBM.  ``value`` is iterations per second
(maxiter * steps / elapsed) of the headline precision mode.

Default workload ``deblur1024``: 1024x1024 image deblurring with a 31x31
Gaussian PSF (sigma 2.5, zero boundary, m = n = 2^20), 1% noise, 150
iterations.  It is timed in three modes: BF16-op (the headline: operator
values and inputs in bfloat16, products summed in float, float bases and
vectors; the projected problem, its parameter choice and the pivot divisions
in FP64), FP32 and FP64 plain.  ``equal_error`` compares each mixed mode with
FP64 plain: iterations/s at K, the wall time of a solve that stops at the
first k within 2 % of FP64's smallest error, and the errors at the stopping
index and at K.

The JSON line also carries the roofline of the dominant kernel -- the
half-iteration kernel of the recurrence (one launch per half-iteration), timed
by the library with HIP events on the stream it launches on -- per mode, the
FP64 CPU oracle timed on a bounded sample of the same workload, and as extra
keys the 128x128 tomography workload (CSR, FP32 and FP64, 100 iterations),
the dense 256x256 blur (FP64, 50 iterations, microseconds per iteration) and
what plain streaming reaches on the same device (a device copy and the
library's matrix-vector product at the shape of the basis).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def _kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2409_05239_amd", "csrc")
    files = ["recurrence.hip", "recurrence_impl.hpp", "device_common.hpp", "internal.hpp"]
    files += sorted(f for f in os.listdir(csrc) if f.startswith("recurrence_psf_"))
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
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
    """Algorithmic bytes of one CSR product: values + column indices (16-bit
    when every index fits, as the library stores them: cols <= 65536), row
    pointers, the input vector once and the output once."""
    isz = 2 if cols <= 65536 else 4
    return nnz * (vsz + isz) + 4 * (rows + 1) + esz * cols + esz * rows


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


def _errors(X, x_true, k_done):
    """Relative error ||x_k - x_true|| / ||x_true|| of every iterate, on the
    device (measurement only; X holds one iterate per row)."""
    import torch
    d = X[:k_done].double() - x_true.double()[None, :]
    return (torch.linalg.norm(d, dim=1) / torch.linalg.norm(x_true.double())).cpu().numpy()


def measure(capi, ctx, prob, cfg, prec, K, steps, warmup, grid, dev, sample=None):
    """Times `steps` solves (graph replays) of the workload in one precision
    mode after `warmup`, then one eager solve with the library's phase events.
    Returns ms per solve, iterations/s, the per-k error to x_true, the last
    solve's info, the phase timing, and a solver for shorter runs."""
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    op = capi.make_operator(ctx, prob, capi.PRECISIONS[prec])
    b = torch.tensor(prob.b, dtype=dt, device=dev)
    X = torch.zeros((K, prob.n), dtype=dt, device=dev)
    x = torch.zeros(prob.n, dtype=dt, device=dev)
    xt = torch.tensor(prob.x_true, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def solve(k=K, timing=False, Xk=X):
        return capi.lslu_solve(ctx, op, b, k, reg=cfg["reg"], lam=cfg.get("lam", 0.0),
                               grid=grid, grid_relative=cfg["grid_relative"], X=Xk, x_out=x,
                               timing=timing,
                               pivot_sample=None if sample is None else (sample[0][:2 * k + 1],
                                                                         sample[1]))

    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, _, info = solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    errs = _errors(X, xt, info["k_done"])
    _, _, tinfo = solve(timing=True)
    torch.cuda.synchronize()

    def time_k(k, reps=5):
        """Median wall time of a k-iteration solve (everything a K-iteration
        step does, for k iterations)."""
        Xk = X[:k]
        solve(k, Xk=Xk)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            solve(k, Xk=Xk)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        return sorted(ts)[reps // 2] * 1e3

    return dict(op=op, ms=el / steps * 1e3, iters_per_s=K * steps / el, errs=errs, info=info,
                timing=tinfo["timing"], time_k=time_k, prec=prec)


def roofline_of(prob, K, prec, tm, workload):
    """Roofline object of the half-iteration kernel (the dominant one): its
    algorithmic bytes per launch (recurrence_bytes over the 2K + 1 launches)
    over its average launch time (HIP events the library records on the
    stream it launches on)."""
    esz = 8 if prec == "fp64" else 4
    vsz = {"fp64": 8, "fp32": 4, "bf16op": 2, "fp16op": 2, "fp8op": 1}[prec]
    n_launch = tm["n_recurrence_launches"]
    t_launch = tm["t_recurrence_ms"] * 1e-3 / n_launch
    nbytes = recurrence_bytes(prob, K, vsz, esz) / n_launch
    kname = "k_half_rows" if prob.kind in ("csr", "dense") else "k_half_psf"
    achieved = nbytes / t_launch / 1e9
    return dict(bound="hbm", kernel=f"{kname} (one half-iteration: product, "
                "elimination, pivot)", achieved=round(achieved, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=_load_traffic(kname, workload, prec),
                us_per_launch=round(t_launch * 1e6, 3), bytes_per_launch=int(nbytes),
                launches_per_step=n_launch,
                phase_ms=dict(recurrence=round(tm["t_recurrence_ms"], 4),
                              projected=round(tm["t_projected_ms"], 4),
                              assemble=round(tm["t_assemble_ms"], 4)))


def equal_error(res, ref="fp64", slack=0.02):
    """The comparison the metric names (mixed precision against FP64 plain at
    equal relative error): per mode, iterations/s at K, the first k whose
    error to x_true is within (1 + slack) of FP64's minimum and the wall time
    of a solve that stops there, and the errors at the stopping index and at
    K; "equal" holds where |e_p - e_FP64| <= slack * e_FP64."""
    e64 = res[ref]["errs"]
    target = (1.0 + slack) * float(e64.min())
    out = {"reference": ref, "slack": slack, "target_rel_err": target}
    base = {}
    for p, r in res.items():
        e = r["errs"]
        hit = np.flatnonzero(e <= target)
        k_t = int(hit[0]) + 1 if hit.size else None
        ms_t = r["time_k"](k_t) if k_t else None
        ks = int(r["info"]["k_stop"])
        d = dict(iters_per_s=round(r["iters_per_s"], 2), ms_per_step=round(r["ms"], 4),
                 rel_err_min=float(e.min()), k_min=int(e.argmin()) + 1,
                 k_target=k_t, ms_to_target=None if ms_t is None else round(ms_t, 4),
                 k_stop=ks, rel_err_at_k_stop=float(e[ks - 1]), rel_err_at_K=float(e[-1]))
        if p == ref:
            base = d
        out[p] = d
    for p, d in out.items():
        if not isinstance(d, dict) or p == ref:
            continue
        d["speedup_iters_per_s"] = round(d["iters_per_s"] / base["iters_per_s"], 4)
        if d["ms_to_target"] and base["ms_to_target"]:
            d["speedup_to_target"] = round(base["ms_to_target"] / d["ms_to_target"], 4)
        e_ks = base["rel_err_at_k_stop"]  # each mode at its own stopping index
        d["equal_at_target"] = d["k_target"] is not None
        d["equal_at_k_stop"] = bool(abs(d["rel_err_at_k_stop"] - e_ks) <= slack * e_ks)
        d["equal_at_K"] = bool(abs(d["rel_err_at_K"] - base["rel_err_at_K"])
                               <= slack * base["rel_err_at_K"])
    return out


def run(args):
    import torch

    from paper_2409_05239_amd import capi
    from workloads import CONFIGS, lambda_grid

    cfg = CONFIGS[args.workload]
    prob = cfg["make"]()
    K = args.iters or cfg["iters"]
    head = args.precision or ("bf16op" if args.workload == "deblur1024" else "fp32")
    modes = [head] if args.no_fp64 else list(dict.fromkeys([head, "fp64", "fp32", "bf16op"]))
    grid = lambda_grid()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # The library launches on this stream; every event below is recorded on it.
    stream = torch.cuda.Stream(device=dev)
    ctx = capi.lslu_create(0, stream=stream)

    sample = None
    if args.pivot_sample > 0:  # the sampled-pivot variant (Section 2.2)
        from workloads import pivot_sample_lists
        sample = (pivot_sample_lists(prob.m, prob.n, K, args.pivot_sample, seed=0),
                  args.pivot_sample)

    print(f"[bench] workload={args.workload} m={prob.m} n={prob.n} nnz={prob.nnz} "
          f"K={K} modes={modes}", flush=True)
    if args.calibrate_copy:
        # A plain device copy of known size (256 MiB read + 256 MiB written),
        # used to scale the FETCH_SIZE / WRITE_SIZE counters.
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    res = {}
    for p in modes:
        res[p] = measure(capi, ctx, prob, cfg, p, K, args.steps, args.warmup, grid, dev, sample)
        print(f"[bench] {p}: {res[p]['ms']:.3f} ms/step, min rel err "
              f"{res[p]['errs'].min():.5f} at k={int(res[p]['errs'].argmin()) + 1}", flush=True)
    eq = equal_error(res) if "fp64" in res and len(res) > 1 else None
    h = res[head]
    roof = roofline_of(prob, K, head, h["timing"], args.workload)
    modes_roof = {p: {k: v for k, v in roofline_of(prob, K, p, r["timing"], args.workload).items()
                      if k in ("frac", "us_per_launch", "achieved", "traffic", "phase_ms")}
                  for p, r in res.items()}
    for r in res.values():
        capi.lslu_op_destroy(r["op"])
    capi.lslu_destroy(ctx)
    errs = h["errs"]

    extra = {}
    if args.workload == "deblur1024" and not args.no_extra:
        extra = extra_workloads(capi, dev, args)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, cfg, grid, args.cpu_iters or (10 if prob.n > 1e6 else K), K)

    out = {
        "metric": "Hybrid LSLU iters/s + % HBM roofline, mixed vs FP64 plain at equal rel. error",
        "value": round(h["iters_per_s"], 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16op": "bf16-op/f32", "fp16op": "f16-op/f32",
                  "fp8op": "f8-op/f32"}[head],
        "data": "synthetic",
        "config": {"workload": args.workload, "m": prob.m, "n": prob.n,
                   "nnz": prob.nnz, "iters": K, "precision": head,
                   "reg": cfg["reg"], "grid_relative": cfg["grid_relative"],
                   "pivot_sample": args.pivot_sample or None},
        "rel_err_final": float(errs[-1]),
        "rel_err_min": float(errs.min()),
        "k_min": int(errs.argmin()) + 1,
        "k_stop": int(h["info"]["k_stop"]),
        "status": int(h["info"]["status"]),
        "equal_error": eq,
        "modes_roofline": modes_roof,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


def extra_workloads(capi, dev, args):
    """The other measured workloads, as extra keys of the JSON line:
    tomography (128^2, CSR, 100 iterations) in FP32 and FP64, and the dense
    256 x 256 blur (50 iterations, FP64) in microseconds per iteration, for
    LSLU (lambda = 0) and Hybrid LSLU (weighted GCV), beside the launch floor
    (microseconds per launch of the same solve on a 64 x 64 problem)."""
    import torch

    from workloads import CONFIGS, lambda_grid
    grid = lambda_grid()
    out = {}
    stream = torch.cuda.Stream(device=dev)
    ctx = capi.lslu_create(0, stream=stream)
    try:
        cfg = CONFIGS["tomo128"]
        prob = cfg["make"]()
        K = cfg["iters"]
        tomo = {}
        for p in ("fp32", "fp64"):
            r = measure(capi, ctx, prob, cfg, p, K, args.steps, args.warmup, grid, dev)
            rf = roofline_of(prob, K, p, r["timing"], "tomo128")
            tomo[p] = dict(iters_per_s=round(r["iters_per_s"], 2), ms_per_step=round(r["ms"], 4),
                           rel_err_min=float(r["errs"].min()), k_min=int(r["errs"].argmin()) + 1,
                           rel_err_at_K=float(r["errs"][-1]), roofline_frac=rf["frac"],
                           us_per_launch=rf["us_per_launch"], traffic=rf["traffic"])
            capi.lslu_op_destroy(r["op"])
            print(f"[bench] tomo128 {p}: {r['ms']:.3f} ms/step", flush=True)
        out["tomo128"] = dict(m=prob.m, n=prob.n, nnz=prob.nnz, iters=K, **tomo)
        cfg = CONFIGS["dense256"]
        prob = cfg["make"]()
        K = cfg["iters"]
        dense = {}
        for reg in ("none", "wgcv"):
            c2 = dict(cfg, reg=reg)
            r = measure(capi, ctx, prob, c2, "fp64", K, max(args.steps, 20), args.warmup, grid,
                        dev)
            tm = r["timing"]
            dense[reg] = dict(us_per_iter=round(r["ms"] * 1e3 / K, 3),
                              us_per_launch=round(tm["t_recurrence_ms"] * 1e3
                                                  / tm["n_recurrence_launches"], 3),
                              rel_err_min=float(r["errs"].min()))
            capi.lslu_op_destroy(r["op"])
            print(f"[bench] dense256 {reg}: {r['ms'] * 1e3 / K:.2f} us/iter", flush=True)
        # the launch floor: the same solve on a 64 x 64 dense problem, whose
        # launches do almost no work
        from workloads import random_dense
        tiny = random_dense(64, 64, seed=7, nu=0.01)
        r = measure(capi, ctx, tiny, dict(cfg, reg="none"), "fp64", K, max(args.steps, 20),
                    args.warmup, grid, dev)
        tm = r["timing"]
        dense["launch_floor_us"] = round(tm["t_recurrence_ms"] * 1e3
                                         / tm["n_recurrence_launches"], 3)
        capi.lslu_op_destroy(r["op"])
        print(f"[bench] launch floor (64 x 64 dense): {dense['launch_floor_us']:.2f} us/launch",
              flush=True)
        out["dense256"] = dict(iters=K, precision="fp64", **dense)
    finally:
        capi.lslu_destroy(ctx)
    out["stream_reference"] = stream_reference(dev)
    return out


def stream_reference(dev, n=1 << 20, k=150, reps=20):
    """What plain streaming reaches on this device, beside the roofline's
    published peak: a 1 GiB device copy (bytes read + written) and the
    library's matrix-vector product over an n x k column-major FP32 matrix,
    the shape of the basis the elimination reads at 1024^2 and 150
    iterations (bytes of the matrix)."""
    import torch

    def timed(f):
        f()
        torch.cuda.synchronize(dev)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            f()
        t1.record()
        torch.cuda.synchronize(dev)
        return t0.elapsed_time(t1) * 1e-3 / reps

    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    copy = 2 * src.numel() * 4 / timed(lambda: dst.copy_(src)) / 1e9
    del src, dst
    basis = torch.ones(k, n, dtype=torch.float32, device=dev)  # column j contiguous
    coef = torch.ones(k, dtype=torch.float32, device=dev)
    gemv = basis.numel() * 4 / timed(lambda: torch.mv(basis.t(), coef)) / 1e9
    del basis, coef
    ref = dict(copy_GBps=round(copy, 1), gemv_GBps=round(gemv, 1),
               gemv_shape=f"{n} x {k} fp32 column-major", peak_GBps=HBM_PEAK_GBS)
    print(f"[bench] stream reference: copy {copy:.0f} GB/s, gemv {gemv:.0f} GB/s", flush=True)
    return ref


def cpu_baseline(prob, cfg, grid, iters, K):
    """The FP64 oracle (as is) on the first ``iters`` iterations of the same
    workload, single-threaded BLAS; iterations per second."""
    from threadpoolctl import threadpool_limits

    from oracle import RegParam, make_operator
    from oracle.hessenberg import hybrid_lslu

    op = make_operator(prob)
    reg = RegParam(cfg["reg"], lam=cfg.get("lam", 0.0), grid=grid,
                   grid_relative=cfg["grid_relative"])
    runs = 1 if iters < K else 3
    times = []
    with threadpool_limits(limits=1):
        for _ in range(runs):
            t0 = time.perf_counter()
            hybrid_lslu(op, prob.b, iters, reg)
            times.append(time.perf_counter() - t0)
    el = sorted(times)[len(times) // 2]
    what = ("the whole solve" if iters >= K else
            f"the first {iters} of {K} iterations (later iterations eliminate more "
            "basis vectors, so this overstates the oracle's rate over the whole solve)")
    try:
        host_cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        host_cores = os.cpu_count()
    return {"value": round(iters / el, 3), "unit": "iters/s", "cores": 1,
            "host_cores": host_cores, "kind": "oracle",
            "sample": f"{what} of the same workload, {'median of 3 runs' if runs > 1 else 'one run'} "
                      f"of {el:.2f} s (FP64 NumPy/SciPy, one thread)"}


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
    value: all problems on S contexts (one stream each), assigned longest
    first to the least loaded context and solved back to back by one host
    thread per context; also timed as asynchronous solves in waves of S.
    Also timed: the same one at a time, FP64 one at a time, and for the
    tomography (CSR) half alone the merged batch
    (lslu_solve_batch: each recurrence launch covers every problem) against
    waves on S contexts and one at a time.  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2409_05239_amd import capi
    from workloads import batch_problems, lambda_grid

    P, S, K = args.batch, args.contexts, 60
    probs = batch_problems(P, seed=0)
    print(f"[batch] {P} problems generated", flush=True)
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

    def cost(prob):
        # rough work per iteration: the operator's products and the basis
        # passes (PSF: taps per pixel over the 16 products a matrix-core
        # instruction forms)
        work = prob.nnz if prob.kind == "csr" else prob.n * prob.psf.size / 16
        return 2 * work + (prob.m + prob.n) * K / 2

    def prepare_lpt(prec, ctxs, sel):
        # longest first onto the least loaded context: each context's
        # problems then run back to back on its own stream (one host thread
        # per context), with no wave boundaries
        order = sorted(range(len(sel)), key=lambda i: -cost(sel[i]))
        load = [0.0] * len(ctxs)
        lists = [[] for _ in ctxs]
        for i in order:
            j = min(range(len(ctxs)), key=lambda q: load[q])
            lists[j].append(i)
            load[j] += cost(sel[i])
        dt = torch.float64 if prec == "fp64" else torch.float32
        items = [None] * len(sel)
        for j, lst in enumerate(lists):
            for i in lst:
                prob = sel[i]
                op = capi.make_operator(ctxs[j], prob, capi.PRECISIONS[prec])
                items[i] = (ctxs[j], op, torch.tensor(prob.b, dtype=dt, device=dev),
                            torch.zeros((K, prob.n), dtype=dt, device=dev))
        torch.cuda.synchronize()
        return items, lists

    def threaded(arg):
        import threading
        items, lists = arg

        def worker(lst):
            for i in lst:
                solve(items[i])

        ths = [threading.Thread(target=worker, args=(lst,)) for lst in lists]
        for t in ths:
            t.start()
        for t in ths:
            t.join()

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
    print(f"[batch] concurrent on {S} contexts: {t_conc * 1e3:.3f} ms", flush=True)
    t_seq = timed(one_at_a_time, lo)
    print(f"[batch] one at a time: {t_seq * 1e3:.3f} ms", flush=True)
    errs = errors(lo, probs)
    release(lo)
    lt = prepare_lpt("bf16op", rr, probs)
    t_thr = timed(threaded, lt)
    print(f"[batch] longest first on {S} contexts, one thread each: {t_thr * 1e3:.3f} ms",
          flush=True)
    errs_thr = errors(lt[0], probs)
    release(lt[0])
    hi = prepare("fp64", rr, probs)
    t_64 = timed(one_at_a_time, hi)
    print(f"[batch] fp64 one at a time: {t_64 * 1e3:.3f} ms", flush=True)
    errs64 = errors(hi, probs)
    release(hi)
    tomo = [p for p in probs if p.kind == "csr"]
    own = [capi.lslu_create(0) for _ in tomo]  # the merged batch: one context each
    mo = prepare("bf16op", own, tomo)
    t_tm = timed(merged, mo)
    print(f"[batch] tomography merged: {t_tm * 1e3:.3f} ms", flush=True)
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
        "value": round(it_total / t_thr, 1),
        "unit": "problem-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_thr * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-op/f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {P} uneven problems (tomography 32-96, deblur 64-256)",
                   "iters": K, "contexts": S, "reg": "wgcv", "grid_relative": True},
        "schedule": "longest first onto the least loaded context, one host thread per "
                    "context solving its problems back to back",
        "same_errors_as_waves": bool(errs_thr == errs),
        "waves": {"value": round(it_total / t_conc, 1), "ms_per_step": round(t_conc * 1e3, 3)},
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
    ap.add_argument("--workload", default="deblur1024")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--cpu-iters", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="time only the headline precision (no equal-error comparison)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the tomography and dense workloads' extra keys")
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
