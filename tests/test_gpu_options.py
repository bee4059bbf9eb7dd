"""GPU: the solve options that change what is formed or reported, against
the oracle and against the library's default solve.

* final-only assembly: only the returned iterate x_out = x_0 + L_k y_k is
  formed (Algorithm 5 forms every x_k; a caller that wants only the result
  needs one of them);
* pivot separations: (a1 - a2)/a1 of every infinity-norm pivot search
  (Algorithm 4), as the oracle records them.
"""

import numpy as np
import pytest

from gpu_helpers import TAU, TOL, pivot_prefix, rel, torch_dtype
from oracle import RegParam, make_operator
from oracle.hessenberg import hybrid_lslu
from workloads import config_problem, lambda_grid, random_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.lslu_create(0)
    yield c
    lib.lslu_destroy(c)


def _solve(lib, ctx, op, prob, prec, K, **kw):
    import torch
    dt = torch_dtype(prec)
    b = torch.tensor(prob.b, dtype=dt, device="cuda")
    x0 = kw.pop("x0", None)
    x0t = None if x0 is None else torch.tensor(x0, dtype=dt, device="cuda")
    st, x, info = lib.lslu_solve(ctx, op, b, K, reg="wgcv", grid=lambda_grid(),
                                 grid_relative=True, x0=x0t, **kw)
    torch.cuda.synchronize()
    info["x"] = x.double().cpu().numpy()
    return info


@pytest.mark.parametrize("name,prec,K", [("dense256", "fp64", 30), ("tomo32", "fp32", 40),
                                         ("deblur96", "fp64", 40), ("deblur96", "fp32", 40)])
@pytest.mark.parametrize("early", [False, True])
def test_final_only_matches_all_iterates(lib, ctx, name, prec, K, early):
    """x_out of a final-only solve equals the default solve's x_out (the
    same iterate, summed in another order: within 4 k u relative in FP64,
    one float rounding in FP32) and, in FP64, the oracle's x_k at the same
    k; every other output is bit-identical."""
    import torch
    prob = config_problem(name)
    op = lib.make_operator(ctx, prob, lib.PRECISIONS[prec])
    rng = np.random.default_rng(5)
    x0 = 0.1 * rng.standard_normal(prob.n)
    try:
        print(f"[final_only] {name} {prec} K={K} early={early}", flush=True)
        kw = dict(early_stop=early, stop_tol=1e-3, x0=x0)
        full = _solve(lib, ctx, op, prob, prec, K, **dict(kw))
        fin = _solve(lib, ctx, op, prob, prec, K, final_only=True, **dict(kw))
        with pytest.raises(ValueError):
            lib.lslu_solve(ctx, op, torch.zeros(prob.m, dtype=torch_dtype(prec), device="cuda"),
                           K, final_only=True,
                           X=torch.zeros((K, prob.n), dtype=torch_dtype(prec), device="cuda"))
    finally:
        lib.lslu_op_destroy(op)
    for key in ("piv_t", "piv_g", "H", "W", "Y", "lambda_idx", "ghat"):
        assert np.array_equal(full[key], fin[key]), key
    assert full["k_stop"] == fin["k_stop"] and full["k_done"] == fin["k_done"]
    ks = fin["k_stop"] if early else fin["k_done"]
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    bound = 4 * ks * u if prec == "fp64" else 2 * u
    d = np.abs(fin["x"] - full["x"]).max() / np.abs(full["x"]).max()
    print(f"[final_only] k_sel {ks}: max difference to the default solve {d:.2e}")
    assert d <= bound, (d, bound)
    # FP64: the oracle's x_k at the same k (same pivots and lambda there)
    if prec == "fp64":
        R = hybrid_lslu(make_operator(prob), prob.b, ks,
                        RegParam("wgcv", grid=lambda_grid(), grid_relative=True), x0=x0)
        assert list(fin["piv_g"][:ks]) == R.piv_g[:ks]
        assert fin["lambda_idx"][ks - 1] == R.lambda_idx[ks - 1]
        e = rel(fin["x"], R.X[:, ks - 1])
        print(f"[final_only] oracle x_{ks}: {e:.2e}")
        assert e <= TOL[prec], e


def _seps(R):
    return np.asarray(R.sep_t), np.asarray(R.sep_g)


@pytest.mark.parametrize("name,K,sampled", [("dense256", 30, False), ("tomo32", 40, False),
                                            ("deblur96", 30, False), ("tomo32", 30, True)])
def test_pivot_separations_match_oracle(lib, ctx, name, K, sampled):
    """FP64: the separation of every search equals the oracle's on the
    prefix where the two chose the same pivots.  The library evaluates it as
    1 - max |v(j)| off the pivot row of the normalised vector v (d_k or
    l_k), the oracle as (a1 - a2)/a1 of the unnormalised one; 1 - max|v| is
    1-Lipschitz in the max norm of v, so the two differ by at most the
    largest entry difference of the two bases' vector plus a few roundings."""
    from workloads import pivot_sample_lists
    prob = config_problem(name)
    ps = None
    if sampled:
        s = 25
        ps = (pivot_sample_lists(prob.m, prob.n, K, s, seed=11), s)
    R = hybrid_lslu(make_operator(prob), prob.b, K,
                    RegParam("wgcv", grid=lambda_grid(), grid_relative=True), pivot_sample=ps)
    op = lib.make_operator(ctx, prob, lib.PRECISIONS["fp64"])
    try:
        print(f"[pivot_sep] {name} K={K} sampled={sampled}", flush=True)
        G = _solve(lib, ctx, op, prob, "fp64", K, pivot_sep=True, pivot_sample=ps)
        plain = _solve(lib, ctx, op, prob, "fp64", K, pivot_sample=ps)
        Lg, Dg = _bases(lib, ctx, prob, G)
    finally:
        lib.lslu_op_destroy(op)
    assert np.array_equal(G["x"], plain["x"])  # the option changes no result
    st, sg = _seps(R)
    k = pivot_prefix(R, TAU["fp64"], min(R.k_done, G["k_done"]))
    assert k >= 5
    # searches t(1), g(1), ..., t(k), g(k) chose the same rows
    assert np.array_equal(G["piv_t"][:k], R.piv_t[:k])
    assert np.array_equal(G["piv_g"][:k], R.piv_g[:k])
    # search t(j) produced d_j, search g(j) produced l_j
    vt = np.abs(Dg[:, :k] - R.D[:, :k]).max(axis=0) + 4 * 2.0 ** -53
    vg = np.abs(Lg[:, :k] - R.L[:, :k]).max(axis=0) + 4 * 2.0 ** -53
    dt = np.abs(G["sep_t"][:k] - st[:k])
    dg = np.abs(G["sep_g"][:k] - sg[:k])
    print(f"[pivot_sep] {name}: {k} iterations compared, max difference "
          f"{max(dt.max(), dg.max()):.2e} (largest basis entry difference "
          f"{max(vt.max(), vg.max()):.2e}); smallest separation "
          f"{min(st[:k].min(), sg[:k].min()):.2e}")
    assert np.all(dt <= vt) and np.all(dg <= vg), (dt.max(), dg.max())
    assert max(vt.max(), vg.max()) <= TOL["fp64"]
    kd = G["k_done"]
    assert np.all((G["sep_t"][:kd] >= 0) & (G["sep_t"][:kd] <= 1))
    assert np.all((G["sep_g"][:kd] >= 0) & (G["sep_g"][:kd] <= 1))


def _bases(lib, ctx, prob, G):
    import torch
    out = []
    for which, cnt, length in ((0, G["n_l"], prob.n), (1, G["n_d"], prob.m)):
        buf = torch.zeros((max(cnt, 1), length), dtype=torch.float64, device="cuda")
        lib.lslu_get_basis(ctx, which, cnt, buf)
        torch.cuda.synchronize()
        out.append(buf.cpu().numpy().T[:, :cnt].copy())
    return out


def test_pivot_separations_of_searches_not_made(lib, ctx):
    """A breakdown at k = 1 on the u side (A = 2 I: u = 2 l_1 - H(1,1) d_1 = 0):
    sep_t(1) and sep_g(1) exist, the searches after it do not (NaN); a
    single candidate gives 1."""
    from workloads.problems import Problem
    n = 6
    A = 2.0 * np.eye(n)
    b = np.array([0.5, -3.0, 1.0, 2.0, 0.0, 1.5])
    prob = Problem("scaled_identity", "dense", n, n, b / 2, b, 0.0, A=A)
    op = lib.make_operator(ctx, prob, lib.PRECISIONS["fp64"])
    try:
        G = _solve(lib, ctx, op, prob, "fp64", 3, pivot_sep=True)
    finally:
        lib.lslu_op_destroy(op)
    assert G["status"] == lib.LSLU_BREAKDOWN_U and G["k_done"] == 1
    R = hybrid_lslu(make_operator(prob), prob.b, 3, RegParam("wgcv", grid=lambda_grid(),
                                                             grid_relative=True))
    st, sg = _seps(R)
    assert len(st) == 1 and len(sg) == 1
    assert abs(G["sep_t"][0] - st[0]) <= 1e-15 and abs(G["sep_g"][0] - sg[0]) <= 1e-15
    assert np.all(np.isnan(G["sep_t"][1:])) and np.all(np.isnan(G["sep_g"][1:]))
    # one candidate: a 1 x 1 problem
    one = random_dense(1, 1, seed=2)
    op = lib.make_operator(ctx, one, lib.PRECISIONS["fp64"])
    try:
        G = _solve(lib, ctx, op, one, "fp64", 1, pivot_sep=True)
    finally:
        lib.lslu_op_destroy(op)
    assert G["sep_t"][0] == 1.0 and G["sep_g"][0] == 1.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", ["dense230x215_K200", "dense60x45_K17", "psf45x77_K140",
                                   "psf8x8_K1"])
def test_iterates_are_basis_times_projected_solutions(lib, ctx, prec, shape):
    """Every x_k = x_0 + L_k y_k (Algorithm 5), checked against the product
    of the library's own L and Y in FP64 on the host, entry by entry, within
    the rounding bound of a k-term FP64 sum (4 k u |x_0| + |L||y_k|) plus the
    storage rounding of x_k.  The shapes take both basis layouts (row-major
    for dense, column-major for PSF), one and two groups of 128 iterates,
    ragged row blocks, odd n (unaligned columns of X) and K = 1."""
    from workloads import psf_deblur
    rng = np.random.default_rng(17)
    if shape.startswith("dense"):
        m, n, K = {"dense230x215_K200": (230, 215, 200), "dense60x45_K17": (60, 45, 17)}[shape]
        prob = random_dense(m, n, seed=21, nu=0.01)
    else:
        side, cols, K = {"psf45x77_K140": (45, 77, 140), "psf8x8_K1": (8, 8, 1)}[shape]
        prob = psf_deblur(side, 3, 1.5, 0.01, seed=22, cols=cols)
    x0 = rng.standard_normal(prob.n)
    G = _gpu(lib, ctx, prob, prec, K, x0)
    kd = G["k_done"]
    assert kd >= min(K, 17)
    L, Y = G["L"][:, :kd], G["Y"][:kd, :kd]
    Xr = x0[:, None] + L @ Y
    if prec == "fp32":
        Xr = x0.astype(np.float32).astype(np.float64)[:, None] + L @ Y
    u = 2.0 ** -53
    bound = 4 * kd * u * (np.abs(x0)[:, None] + np.abs(L) @ np.abs(Y))
    if prec == "fp32":
        bound += 2.0 ** -24 * np.abs(Xr)
    err = np.abs(G["X"][:, :kd] - Xr)
    print(f"[assembly] {shape} {prec} k_done {kd}: max |X - (x0 + L Y)| {err.max():.2e}, "
          f"max ratio to the bound {(err / (bound + 1e-300)).max():.2f}")
    assert np.all(err <= bound + 1e-300)


def _gpu(lib, ctx, prob, prec, K, x0):
    from gpu_helpers import gpu_solve
    return gpu_solve(lib, ctx, prob, prec, K, "wgcv", grid=lambda_grid(), grid_relative=True,
                     x0=x0)
