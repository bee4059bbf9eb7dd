"""Many problems at once: asynchronous solves on several contexts (one stream
each) against the same solves run one at a time.

Every problem's results must be bit-identical however the solves are
interleaved: the kernels of one solve depend only on that solve's data, and
the waits inside a launch only ever wait for blocks of the same launch that
were dispatched before the waiting block.
"""

import numpy as np
import pytest

from workloads import batch_problems, lambda_grid

pytestmark = pytest.mark.gpu

K = 20


def _prepare(lib, ctxs, probs, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    items = []
    for i, prob in enumerate(probs):
        c = ctxs[i % len(ctxs)]
        op = lib.make_operator(c, prob, lib.PRECISIONS[prec])
        b = torch.tensor(prob.b, dtype=dt, device="cuda")
        X = torch.zeros((K, prob.n), dtype=dt, device="cuda")
        items.append((c, op, b, X))
    torch.cuda.synchronize()
    return items


def _solve(lib, item, asynchronous=False):
    c, op, b, X = item
    return lib.lslu_solve(c, op, b, K, reg="wgcv", grid=lambda_grid(), grid_relative=True,
                          X=X, asynchronous=asynchronous)


@pytest.mark.parametrize("prec", ["fp32", "bf16op", "fp8op"])
def test_concurrent_solves_match_one_at_a_time(lib, prec):
    import torch
    probs = batch_problems(8, seed=3)
    ctxs = [lib.lslu_create(0) for _ in range(4)]
    try:
        items = _prepare(lib, ctxs, probs, prec)
        print(f"[batch] {prec}: " + ", ".join(p.name for p in probs), flush=True)
        ref = []
        for it in items:  # one at a time, synchronous
            st, x, info = _solve(lib, it)
            ref.append((info, it[3].clone()))
        torch.cuda.synchronize()
        for rep in range(2):  # all contexts busy at once, twice
            out = [None] * len(items)
            for w in range(0, len(items), len(ctxs)):
                wave = list(range(w, min(w + len(ctxs), len(items))))
                pend = {i: _solve(lib, items[i], asynchronous=True) for i in wave}
                for i in wave:
                    st, x, info = lib.lslu_wait(items[i][0], pend[i])
                    out[i] = (info, items[i][3].clone())
            torch.cuda.synchronize()
            for (ri, rX), (oi, oX) in zip(ref, out):
                assert oi["k_done"] == ri["k_done"]
                assert np.array_equal(oi["piv_t"], ri["piv_t"])
                assert np.array_equal(oi["piv_g"], ri["piv_g"])
                assert np.array_equal(oi["H"], ri["H"])
                assert torch.equal(oX, rX)
        for c, op, b, X in items:
            lib.lslu_op_destroy(op)
    finally:
        for c in ctxs:
            lib.lslu_destroy(c)


def test_pending_solve_rules(lib):
    import torch
    probs = batch_problems(2, seed=5)
    c = lib.lslu_create(0)
    try:
        items = _prepare(lib, [c], probs, "fp32")
        # nothing pending: waiting is a no-op
        assert lib.lib.lslu_wait(c) == lib.LSLU_OK
        pend = _solve(lib, items[0], asynchronous=True)
        # a second solve, or a basis copy, while one is pending is refused
        with pytest.raises(lib.LsluError) as ei:
            _solve(lib, items[1])
        assert ei.value.status == lib.LSLU_EINVAL
        dst = torch.zeros((1, probs[0].n), dtype=torch.float32, device="cuda")
        with pytest.raises(lib.LsluError):
            lib.lslu_get_basis(c, 0, 1, dst)
        st, x, info = lib.lslu_wait(c, pend)
        assert info["k_done"] == K
        # timing needs a synchronous solve
        with pytest.raises(lib.LsluError):
            cc, op, b, X = items[1]
            lib.lslu_solve(cc, op, b, K, reg="wgcv", grid=lambda_grid(), grid_relative=True,
                           X=X, asynchronous=True, timing=True)
        for _, op, _, _ in items:
            lib.lslu_op_destroy(op)
    finally:
        lib.lslu_destroy(c)


def _tomo_set(count, seed):
    from workloads import tomography
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(rng.integers(20, 49))
        out.append(tomography(side, side, side + 1, 0.02, seed=seed * 1000 + i))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16op", "fp8op", "fp64"])
def test_merged_launch_batch_matches_single_solves(lib, prec):
    """lslu_solve_batch runs launch j of every problem's recurrence in one
    kernel launch: each problem's results must equal its solve alone."""
    import torch
    from workloads import random_dense
    probs = _tomo_set(6, 7) if prec != "fp64" else [random_dense(60 + 7 * i, 40 + 3 * i, seed=i)
                                                    for i in range(5)]
    dt = torch.float64 if prec == "fp64" else torch.float32
    ctxs = [lib.lslu_create(0) for _ in probs]
    ops = []
    try:
        for c, prob in zip(ctxs, probs):
            ops.append(lib.make_operator(c, prob, lib.PRECISIONS[prec]))
        bs = [torch.tensor(p.b, dtype=dt, device="cuda") for p in probs]
        grid = lambda_grid()
        print(f"[batch] merged {prec}: " + ", ".join(p.name for p in probs), flush=True)
        st, out = lib.lslu_solve_batch(ctxs, ops, bs, K, reg="wgcv", grid=grid, grid_relative=True)
        torch.cuda.synchronize()
        for i, (c, op, b) in enumerate(zip(ctxs, ops, bs)):
            st1, x1, i1 = lib.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True)
            torch.cuda.synchronize()
            xb, ib = out[i]
            assert ib["k_done"] == i1["k_done"], i
            assert np.array_equal(ib["piv_t"], i1["piv_t"]) and np.array_equal(ib["piv_g"], i1["piv_g"])
            assert np.array_equal(ib["H"], i1["H"]) and np.array_equal(ib["lambda_k"], i1["lambda_k"])
            assert torch.equal(xb, x1), i
        # a second batch on the same contexts reuses their workspaces
        st2, out2 = lib.lslu_solve_batch(ctxs, ops, bs, K, reg="wgcv", grid=grid, grid_relative=True)
        torch.cuda.synchronize()
        for (xa, ia), (xb2, ib2) in zip(out, out2):
            assert torch.equal(xa, xb2) and np.array_equal(ia["H"], ib2["H"])
    finally:
        for op in ops:
            lib.lslu_op_destroy(op)
        for c in ctxs:
            lib.lslu_destroy(c)


def test_merged_launch_batch_rejects_what_it_cannot_merge(lib):
    import torch
    from workloads import psf_deblur, random_dense
    probs = [random_dense(30, 20, seed=1), psf_deblur(16, 2, 1.0, 0.01, seed=2)]
    ctxs = [lib.lslu_create(0) for _ in range(3)]
    ops = []
    try:
        ops = [lib.make_operator(ctxs[0], probs[0], lib.LSLU_FP64),
               lib.make_operator(ctxs[1], probs[1], lib.LSLU_FP64),
               lib.make_operator(ctxs[2], probs[0], lib.LSLU_FP32)]
        # a well-formed b for each operator, so the library itself refuses
        bs = [torch.tensor(probs[0].b, dtype=torch.float64, device="cuda"),
              torch.tensor(probs[1].b, dtype=torch.float64, device="cuda"),
              torch.tensor(probs[0].b, dtype=torch.float32, device="cuda")]
        for sel in ([0, 1], [0, 2]):  # a PSF operator; mixed precisions
            with pytest.raises(lib.LsluError) as ei:
                lib.lslu_solve_batch([ctxs[i] for i in sel], [ops[i] for i in sel],
                                     [bs[i] for i in sel], 5)
            assert ei.value.status == lib.LSLU_EINVAL
        op_b = lib.make_operator(ctxs[0], probs[0], lib.LSLU_FP64)
        ops.append(op_b)
        with pytest.raises(lib.LsluError):  # two problems on one context
            lib.lslu_solve_batch([ctxs[0], ctxs[0]], [ops[0], op_b], [bs[0], bs[0]], 5)
    finally:
        for op in ops:
            lib.lslu_op_destroy(op)
        for c in ctxs:
            lib.lslu_destroy(c)


def test_merged_launch_batch_early_stop(lib):
    """The stopping rule and the early-stop iterate of a merged batch equal
    those of single solves."""
    import torch
    probs = _tomo_set(4, 9)
    ctxs = [lib.lslu_create(0) for _ in probs]
    ops = []
    try:
        for c, prob in zip(ctxs, probs):
            ops.append(lib.make_operator(c, prob, lib.PRECISIONS["fp32"]))
        bs = [torch.tensor(p.b, dtype=torch.float32, device="cuda") for p in probs]
        grid = lambda_grid()
        st, out = lib.lslu_solve_batch(ctxs, ops, bs, K, reg="wgcv", grid=grid,
                                       grid_relative=True, stop_tol=1e-3, early_stop=True)
        torch.cuda.synchronize()
        for i, (c, op, b) in enumerate(zip(ctxs, ops, bs)):
            st1, x1, i1 = lib.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True,
                                         stop_tol=1e-3, early_stop=True)
            torch.cuda.synchronize()
            xb, ib = out[i]
            assert ib["k_stop"] == i1["k_stop"] and torch.equal(xb, x1), i
    finally:
        for op in ops:
            lib.lslu_op_destroy(op)
        for c in ctxs:
            lib.lslu_destroy(c)


def _oracle_checks(prob, info, x, prec, K):
    """One batched problem against the FP64 oracle run alone: FP64 -- pivots
    over the oracle's well-separated prefix, and where that prefix covers the
    whole solve, H, W, the lambda indices, Ghat and the final iterate; the
    low-precision modes -- the error to x_true at K against the oracle's."""
    from gpu_helpers import TAU, check_ghat, pivot_prefix, rel, well_separated_prefix
    from oracle import RegParam, make_operator
    from oracle.hessenberg import hybrid_lslu
    from sensitivity import measured_prefix
    reg = RegParam("wgcv", grid=lambda_grid(), grid_relative=True)
    R = hybrid_lslu(make_operator(prob), prob.b, K, reg)
    xg = x.double().cpu().numpy()
    if prec != "fp64":
        # no x-parity requirement in the low-precision operator modes (their
        # products are pinned by test_gpu_parity.test_operator_products): the
        # error to x_true at K is stated against the oracle's, and only a
        # gross departure (a wrong operator, a broken solve) fails here
        e_g, e_r = rel(xg, prob.x_true), rel(R.x, prob.x_true)
        print(f"[batch oracle] {prob.name} {prec}: err at K {e_g:.4f} (fp64 oracle {e_r:.4f})")
        assert np.isfinite(e_g) and e_g <= 1.5 * e_r, (prob.name, e_g, e_r)
        return
    kd = min(R.k_done, info["k_done"])
    kp = pivot_prefix(R, TAU["fp64"], kd)
    assert list(info["piv_g"][:kp]) == R.piv_g[:kp], prob.name
    assert list(info["piv_t"][:kp]) == R.piv_t[:kp], prob.name
    # the stated 1e-10 holds where the problem's measured sensitivity allows it
    ks = measured_prefix(prob, R, reg, kd, 2.0 ** -53, 1e-10)
    k_ok = min(well_separated_prefix(R, TAU["fp64"], kd), ks)
    # H and W depend on the pivots only (not on lambda)
    kh = min(kp, ks)
    Hs, Ws = np.abs(R.H).max(), np.abs(R.W).max()
    if kh > 0:
        assert np.abs(info["H"][:kh + 1, :kh] - R.H[:kh + 1, :kh]).max() <= 1e-9 * Hs
        assert np.abs(info["W"][:kh, :kh] - R.W[:kh, :kh]).max() <= 1e-9 * Ws
    for k in range(1, k_ok + 1):
        assert info["lambda_idx"][k - 1] == R.lambda_idx[k - 1], (prob.name, k)
        check_ghat(info, R, k, "fp64")
    if k_ok == kd == K:
        assert rel(xg, R.x) <= 1e-10, prob.name
    if kd > ks:
        dH = np.abs(info["H"][:kd + 1, :kd] - R.H[:kd + 1, :kd]).max(axis=0) / Hs
        print(f"[batch oracle] {prob.name}: beyond k = {ks} (k, kappa(H), max |dH|/max|H|): "
              + ", ".join(f"({k}, {np.linalg.cond(R.H[:k + 1, :k]):.0f}, {dH[k - 1]:.1e})"
                          for k in range(ks + 1, kd + 1, 3)))
    print(f"[batch oracle] {prob.name}: pivots equal for k <= {kp}, stated tolerance "
          f"applies for k <= {ks}, separated prefix {k_ok} of {kd}")


@pytest.mark.parametrize("prec", ["fp64", "bf16op"])
def test_batched_solves_match_oracle(lib, prec):
    """Problems of the batched workload's kinds (tomography with side = angles,
    side + 1 bins; deblurring with a Gaussian PSF) solved together --
    tomography through merged launches (lslu_solve_batch), deblurring as
    concurrent solves on their own contexts -- against the FP64 oracle."""
    import torch
    from workloads import psf_deblur
    dt = torch.float64 if prec == "fp64" else torch.float32
    tomo = _tomo_set(4, 11)
    blur = [psf_deblur(s, int(np.ceil(3 * sg)), sg, 0.01, seed=2000 + s)
            for s, sg in ((40, 1.5), (56, 2.5), (48, 4.0))]
    ctxs = [lib.lslu_create(0) for _ in tomo + blur]
    ops = []
    try:
        for c, prob in zip(ctxs, tomo + blur):
            ops.append(lib.make_operator(c, prob, lib.PRECISIONS[prec]))
        bs = [torch.tensor(p.b, dtype=dt, device="cuda") for p in tomo + blur]
        grid = lambda_grid()
        nt = len(tomo)
        print(f"[batch oracle] {prec}: " + ", ".join(p.name for p in tomo + blur), flush=True)
        st, out = lib.lslu_solve_batch(ctxs[:nt], ops[:nt], bs[:nt], K, reg="wgcv", grid=grid,
                                       grid_relative=True)
        pend = [lib.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True,
                               asynchronous=True)
                for c, op, b in zip(ctxs[nt:], ops[nt:], bs[nt:])]
        for c, pd in zip(ctxs[nt:], pend):
            st1, x1, i1 = lib.lslu_wait(c, pd)
            out.append((x1, i1))
        torch.cuda.synchronize()
        for prob, (x, info) in zip(tomo + blur, out):
            _oracle_checks(prob, info, x, prec, K)
    finally:
        for op in ops:
            lib.lslu_op_destroy(op)
        for c in ctxs:
            lib.lslu_destroy(c)


def test_merged_batches_from_several_threads(lib):
    """Merged batches of size classes from several host threads at once, one
    more thread capturing and replaying single solves meanwhile (the library
    call releases the interpreter; no thread's copy may touch the legacy
    stream while another captures): every result equals the problem's solve
    alone."""
    import threading

    import torch
    probs = sorted(_tomo_set(8, 11), key=lambda p: p.m)
    solo_probs = _tomo_set(2, 12)
    grid = lambda_grid()
    ctxs = [lib.lslu_create(0) for _ in probs]
    solo_ctx = lib.lslu_create(0)
    ops, solo_ops = [], []
    try:
        for c, prob in zip(ctxs, probs):
            ops.append(lib.make_operator(c, prob, lib.PRECISIONS["bf16op"]))
        for prob in solo_probs:
            solo_ops.append(lib.make_operator(solo_ctx, prob, lib.PRECISIONS["bf16op"]))
        bs = [torch.tensor(p.b, dtype=torch.float32, device="cuda") for p in probs]
        sbs = [torch.tensor(p.b, dtype=torch.float32, device="cuda") for p in solo_probs]
        torch.cuda.synchronize()
        groups = [list(range(g * 2, g * 2 + 2)) for g in range(4)]  # 4 size classes
        results, errors = {}, []

        # No device-wide synchronisation inside the threads: it would race
        # with the fifth thread's graph capture (the library calls wait for
        # their own streams, and each batch call returns new x tensors).
        def merged(g):
            try:
                for rep in range(2):
                    st, out = lib.lslu_solve_batch([ctxs[i] for i in g], [ops[i] for i in g],
                                                   [bs[i] for i in g], K, reg="wgcv", grid=grid,
                                                   grid_relative=True)
                    for i, (x, info) in zip(g, out):
                        results[(i, rep)] = (x, info)
            except Exception as e:  # reported below, in the test's thread
                errors.append(e)

        def solos():
            try:
                for rep in range(3):  # the first call captures, the others replay
                    for op, b in zip(solo_ops, sbs):
                        lib.lslu_solve(solo_ctx, op, b, K, reg="wgcv", grid=grid,
                                       grid_relative=True)
            except Exception as e:
                errors.append(e)

        print("[batch] merged size classes from 4 threads, single solves on a fifth",
              flush=True)
        ths = [threading.Thread(target=merged, args=(g,)) for g in groups]
        ths.append(threading.Thread(target=solos))
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        torch.cuda.synchronize()
        assert not errors, errors
        for i, (c, op, b) in enumerate(zip(ctxs, ops, bs)):
            st1, x1, i1 = lib.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True)
            torch.cuda.synchronize()
            for rep in range(2):
                xb, ib = results[(i, rep)]
                assert torch.equal(xb, x1), (i, rep)
                assert np.array_equal(ib["piv_t"], i1["piv_t"])
                assert np.array_equal(ib["H"], i1["H"]) and np.array_equal(ib["ghat"], i1["ghat"])
    finally:
        for op in ops + solo_ops:
            lib.lslu_op_destroy(op)
        for c in ctxs + [solo_ctx]:
            lib.lslu_destroy(c)


@pytest.mark.skip(reason="the graph-captured batch (one HIP graph over lane streams with every "
                         "problem's solve and its result copy) was taken out of the library: "
                         "its first capture ended the process with a host segmentation fault "
                         "whose cause was not found; kept as the record of the case")
def test_graph_batch_matches_single_solves(lib):
    """LSLU_FLAG_BATCH_GRAPH: every problem's solve captured into one graph
    over lane streams and replayed; tomography (CSR) and deblurring (PSF)
    problems in two precisions mixed in one batch, more problems than lanes.
    The replays reuse the cached graph; every result equals the problem's
    solve alone, bit for bit."""
    import torch
    probs = batch_problems(12, seed=21)
    precs = ["bf16op" if i % 3 else "fp32" for i in range(len(probs))]
    grid = lambda_grid()
    ctxs = [lib.lslu_create(0) for _ in probs]
    ops = []
    try:
        for c, prob, pr in zip(ctxs, probs, precs):
            ops.append(lib.make_operator(c, prob, lib.PRECISIONS[pr]))
        bs = [torch.tensor(p.b, dtype=torch.float32, device="cuda") for p in probs]
        xo = [torch.zeros(p.n, dtype=torch.float32, device="cuda") for p in probs]
        torch.cuda.synchronize()
        print("[batch] graph: " + ", ".join(f"{p.name}/{pr}" for p, pr in zip(probs, precs)),
              flush=True)
        outs = []
        for rep in range(3):  # the first call captures, the others replay
            xo_rep = [x.zero_() for x in xo]
            st, out = lib.lslu_solve_batch(ctxs, ops, bs, K, reg="wgcv", grid=grid,
                                           grid_relative=True, graph=True, x_outs=xo_rep)
            torch.cuda.synchronize()
            outs.append([(x.clone(), info) for x, info in out])
        for i, (c, op, b) in enumerate(zip(ctxs, ops, bs)):
            st1, x1, i1 = lib.lslu_solve(c, op, b, K, reg="wgcv", grid=grid, grid_relative=True)
            torch.cuda.synchronize()
            for rep in range(3):
                xb, ib = outs[rep][i]
                assert ib["k_done"] == i1["k_done"], (i, rep)
                assert np.array_equal(ib["piv_t"], i1["piv_t"])
                assert np.array_equal(ib["piv_g"], i1["piv_g"])
                assert np.array_equal(ib["H"], i1["H"]) and np.array_equal(ib["ghat"], i1["ghat"])
                assert torch.equal(xb, x1), (i, rep)
        # a single solve refuses the batch-only flag
        with pytest.raises(lib.LsluError) as ei:
            o = lib.lslu_opts()
            o.maxiter = K
            o.flags = lib.LSLU_FLAG_BATCH_GRAPH
            x = torch.zeros(probs[0].n, dtype=torch.float32, device="cuda")
            lib._check(ctxs[0], lib.lib.lslu_solve(ctxs[0], ops[0], lib._dptr(bs[0]), None,
                                                   o, lib._dptr(x), None))
        assert ei.value.status == lib.LSLU_EINVAL
    finally:
        for op in ops:
            lib.lslu_op_destroy(op)
        for c in ctxs:
            lib.lslu_destroy(c)
