"""Helpers for the GPU parity tests: run the HIP library through its C ABI on a
``workloads.Problem`` and compare with the oracle's result."""

from __future__ import annotations

import numpy as np

TAU = {"fp64": 1e-9, "fp32": 1e-3, "bf16op": 1e-2, "fp16op": 1e-2, "fp8op": 1e-1}
TOL = {"fp64": 1e-10, "fp32": 1e-4}


def e4m3(x):
    """Round to the 8-bit E4M3 format in its finite, saturating form: 3
    fraction bits, exponent bias 7 (normal exponents -6..8), subnormal spacing
    2^-9, ties to even, largest finite 448."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    e = np.maximum(np.floor(np.log2(np.where(a > 0, a, 1.0))), -6.0)
    q = 2.0 ** (e - 3)
    r = np.minimum(np.round(a / q) * q, 448.0)  # np.round: half to even
    return np.copysign(np.where(a > 0, r, 0.0), x)


def torch_dtype(prec):
    import torch
    return torch.float64 if prec == "fp64" else torch.float32


def gpu_solve(capi, ctx, prob, prec="fp64", K=10, reg="none", lam=0.0,
              grid=None, grid_relative=False, replay=None, x0=None,
              early_stop=False, stop_tol=0.0, bases=True, op=None, eager=False,
              b=None, x_true=None, pivot_sample=None, grad_lambda=False):
    """Solve on the GPU; returns the info dict with x, X (n x K), L, D."""
    import torch
    dt = torch_dtype(prec)
    own_op = op is None
    if own_op:
        op = capi.make_operator(ctx, prob, capi.PRECISIONS[prec])
    try:
        print(f"[gpu_solve] {prob.name} prec={prec} K={K} reg={reg} "
              f"replay={replay is not None}", flush=True)
        if b is None:
            b = torch.tensor(prob.b, dtype=dt, device="cuda")
        X = torch.zeros((K, prob.n), dtype=dt, device="cuda")
        x0t = None if x0 is None else torch.tensor(x0, dtype=dt, device="cuda")
        xtt = None if x_true is None else torch.tensor(x_true, dtype=dt, device="cuda")
        kw = {}
        if replay is not None:
            kw.update(replay)
        st, x, info = capi.lslu_solve(ctx, op, b, K, reg=reg, lam=lam, grid=grid,
                                      grid_relative=grid_relative, X=X, x0=x0t,
                                      early_stop=early_stop, stop_tol=stop_tol,
                                      eager=eager, x_true=xtt,
                                      pivot_sample=pivot_sample,
                                      grad_lambda=grad_lambda, **kw)
        torch.cuda.synchronize()
        info["x"] = x.double().cpu().numpy()
        info["X"] = X.double().cpu().numpy().T.copy()
        if bases:
            nl, nd = info["n_l"], info["n_d"]
            Lt = torch.zeros((max(nl, 1), prob.n), dtype=dt, device="cuda")
            Dt = torch.zeros((max(nd, 1), prob.m), dtype=dt, device="cuda")
            capi.lslu_get_basis(ctx, 0, nl, Lt)
            capi.lslu_get_basis(ctx, 1, nd, Dt)
            torch.cuda.synchronize()
            info["L"] = Lt.double().cpu().numpy().T[:, :nl].copy()
            info["D"] = Dt.double().cpu().numpy().T[:, :nd].copy()
        return info
    finally:
        if own_op:
            capi.lslu_op_destroy(op)


def replay_from(R, K):
    """Replay arrays (pivots and lambda indices) from an oracle result."""
    pt = np.full(K + 1, -1, np.int32)
    pg = np.full(K, -1, np.int32)
    t = np.asarray(R.piv_t[:K + 1], np.int32)
    g = np.asarray(R.piv_g[:K], np.int32)
    pt[:t.shape[0]] = t
    pg[:g.shape[0]] = g
    li = np.full(K, -1, np.int32)
    lk = np.asarray(R.lambda_idx[:K], np.int32)
    li[:lk.shape[0]] = lk
    return dict(replay_piv_t=pt, replay_piv_g=pg, replay_lambda_idx=li)


def pivot_prefix(R, tau, k_max):
    """Largest k such that the pivot searches t(1), g(1), ..., t(k), g(k) all
    have separation above tau in the oracle (pivots never depend on lambda)."""
    k_ok = 0
    for k in range(1, k_max + 1):
        seps = [R.sep_t[k - 1], R.sep_g[k - 1]] if k - 1 < len(R.sep_g) else []
        if len(seps) < 2 or min(seps) <= tau:
            break
        k_ok = k
    return k_ok


def well_separated_prefix(R, tau, k_max):
    """Largest k such that every search deciding x_1..x_k (the pivots up to
    g(k) and lambda_1..lambda_k) has separation above tau."""
    k_ok = 0
    for k in range(1, pivot_prefix(R, tau, k_max) + 1):
        if k - 1 < len(R.sep_lambda) and R.sep_lambda[k - 1] <= tau:
            break
        k_ok = k
    return k_ok


#: Relative tolerance of Ghat(k) (eq. stop2) where x_k is held to TOL: Ghat is
#: a ratio of the projected residual and a trace, both smooth in H_{k+1,k};
#: the library evaluates the residual/trace form from a bidiagonalisation,
#: the oracle the SVD form, so only rounding separates them.
GHAT_TOL = {"fp64": 1e-8, "fp32": 1e-3}


def check_ghat(G, R, k, prec):
    """Ghat(k) of the library against the oracle's at iteration k."""
    g, r = G["ghat"][k - 1], R.ghat[k - 1]
    assert abs(g - r) <= GHAT_TOL[prec] * abs(r), (k, g, r)


def stated_prefix(H, K, prec):
    """Largest k <= K such that 10 k' u kappa(H_{k'+1,k'}) <= TOL[prec] for
    every k' <= k, from the oracle's H: where rounding of relative size u,
    amplified by the conditioning of the projected problem, stays within the
    stated tolerance.  Beyond it the stated tolerance is not asserted (the
    tests record k, kappa and the error instead)."""
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    for k in range(1, K + 1):
        if 10.0 * k * u * np.linalg.cond(H[:k + 1, :k]) > TOL[prec]:
            return k - 1
    return K


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def residual_gap(op, b, x, x_ref):
    """Difference of the relative residuals ||b - A x|| / ||b|| of two
    iterates."""
    r = np.linalg.norm(b - op.matvec(x))
    r_ref = np.linalg.norm(b - op.matvec(x_ref))
    return abs(r - r_ref) / np.linalg.norm(b)


def check_basis_invariants(info, m, n, bound=1.0):
    """Exact structure of the bases in any precision (unit at own pivot, zero at
    earlier pivots, distinct pivots, H Hessenberg) and |entries| <= bound.
    With its own pivots the library guarantees bound = 1; in replay mode the
    imposed pivot may be a rounding error smaller than the largest entry."""
    L, D = info["L"], info["D"]
    pg = [int(v) for v in info["piv_g"][:info["n_l"]]]
    pt = [int(v) for v in info["piv_t"][:info["n_d"]]]
    assert len(set(pg)) == len(pg) and len(set(pt)) == len(pt)
    for k, g in enumerate(pg):
        assert L[g, k] == 1.0
        for j in range(k):
            assert L[pg[j], k] == 0.0
    for k, t in enumerate(pt):
        assert D[t, k] == 1.0
        for j in range(k):
            assert D[pt[j], k] == 0.0
    assert np.all(np.abs(L) <= bound) and np.all(np.abs(D) <= bound)
    kd = info["k_done"]
    H = info["H"]
    assert np.all(np.tril(H[:kd + 1, :kd], -2) == 0)


def check_relations(info, op, prec):
    """A L_k = D_{k+1} H_{k+1,k} and A^T D_k = L_k W_k (eq. nhr, eq. nhr2) for
    the bases and coefficients the GPU produced, to rounding of the working
    precision."""
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    k = min(info["n_l"], info["n_d"] - 1)
    if k < 1:
        return
    L, D = info["L"][:, :k], info["D"][:, :k + 1]
    H, W = info["H"][:k + 1, :k], info["W"][:k, :k]
    AL = np.stack([op.matvec(L[:, j]) for j in range(k)], axis=1)
    ATD = np.stack([op.rmatvec(D[:, j]) for j in range(k)], axis=1)
    r1 = np.linalg.norm(AL - D @ H)
    s1 = np.linalg.norm(AL) + np.linalg.norm(D) * np.linalg.norm(H)
    r2 = np.linalg.norm(ATD - L @ W)
    s2 = np.linalg.norm(ATD) + np.linalg.norm(L) * np.linalg.norm(W)
    assert r1 <= 10 * k * u * s1, (r1 / s1, k)
    assert r2 <= 10 * k * u * s2, (r2 / s2, k)
