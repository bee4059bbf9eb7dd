"""GPU checks at the full sizes of the measured workloads.

* tomo128 (CSR 32580 x 16384, 100 iterations): the FP64 oracle runs the whole
  solve; the FP32 library follows its pivots and lambda indices (replay) and
  must satisfy the Hessenberg relations at every k; the FP64 library runs
  free and matches the pivots over the well-separated prefix.  x_k is held
  to the stated 1e-4 (FP32) / 1e-10 (FP64) at every k where the problem's
  forward sensitivity allows it -- where 10 k u s_k does not exceed the
  stated value, s_k measured on the oracle alone (``sensitivity.py``);
  beyond, the tests record k, kappa(H_{k+1,k}), s_k and the error (no bound
  is asserted there).
* deblur1024 (31x31 PSF on 1024^2, 150 iterations): element-wise parity
  with the oracle's stored solve is in ``test_gpu_golden1024.py``; here,
  what the oracle can compute piece by piece on the library's own output --
  the exact pivot structure of the bases, the Hessenberg relations at sampled
  pixels (the PSF product of one pixel is a 31x31 neighbourhood sum), the
  projected problem re-solved by the oracle from the library's H and beta,
  x_k at sampled pixels from the library's L and y_k, and bit-identical
  repeats.
"""

import numpy as np
import pytest

from gpu_helpers import (TAU, check_basis_invariants, check_ghat,
                         check_relations, gpu_solve, pivot_prefix, rel,
                         replay_from, residual_gap)
from oracle import RegParam, make_operator
from oracle.hessenberg import hybrid_lslu
from oracle.projected import projected_svd, select_lambda, tikhonov_coeffs
from sensitivity import perturbed_runs, sensitivity_at, step_tolerances
from workloads import config_problem, lambda_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.lslu_create(0)
    yield c
    lib.lslu_destroy(c)


@pytest.fixture(scope="module")
def tomo():
    prob = config_problem("tomo128")
    reg = RegParam("wgcv", grid=lambda_grid(), grid_relative=True)
    R = hybrid_lslu(make_operator(prob), prob.b, 100, reg)
    runs = perturbed_runs(prob, R, reg, 100)
    sens = sensitivity_at(runs, R.lambdas, R.X, min(100, R.k_done))
    return prob, R, sens, runs


def _beyond(tag, K, k_stated, errs, R, sens):
    """Records k, kappa(H_{k+1,k}), s_k and the error where the stated
    tolerance does not apply."""
    rows = []
    for k in list(range(k_stated + 1, K + 1, 8)) + [K]:
        if k > k_stated:
            kap = np.linalg.cond(R.H[:k + 1, :k])
            rows.append(f"({k}, {kap:.0f}, {sens[k - 1]:.1e}, {errs[k - 1]:.1e})")
    print(f"[{tag}] beyond k = {k_stated} (k, kappa(H), s_k, err): " + ", ".join(rows))


def test_tomo128_fp32_replay_full(lib, ctx, tomo):
    """FP32 following the oracle's pivots and lambda indices for 100 steps.

    What holds at any k is the backward-error statement -- the Hessenberg
    relations to FP32 rounding -- and the exact pivot structure.  Forward
    parity with the FP64 oracle is held to the stated 1e-4 wherever the
    problem's forward sensitivity allows it (``sensitivity.py``: the LU-type
    bases of this problem turn a relative perturbation of 1e-9 into ~1e-6 by
    k = 16 and ~3e-5 by k = 79); beyond, k, kappa, s_k and the error are
    recorded."""
    prob, R, sens, _ = tomo
    K = min(100, R.k_done)
    G = gpu_solve(lib, ctx, prob, "fp32", K, "wgcv", grid=lambda_grid(),
                  grid_relative=True, replay=replay_from(R, K))
    # The imposed pivot need not be the FP32 vector's largest entry once the
    # two precisions have drifted apart, so only the exact structure holds.
    check_basis_invariants(G, prob.m, prob.n, bound=np.inf)
    op = make_operator(prob)
    check_relations(G, op, "fp32")
    assert G["k_stop"] == R.k_stop
    tol = step_tolerances(sens[:K], 2.0 ** -24, 1e-4)
    errs = np.array([rel(G["X"][:, k], R.X[:, k]) for k in range(K)])
    gaps = np.array([residual_gap(op, prob.b, G["X"][:, k], R.X[:, k]) for k in range(K)])
    k_stated = int(np.argmax(tol > 1e-4)) if np.any(tol > 1e-4) else K
    print(f"[tomo128 fp32 replay] stated 1e-4 applies for k <= {k_stated}; "
          f"max err there {errs[:k_stated].max():.2e}, max residual gap "
          f"{gaps[:k_stated].max():.2e}")
    assert k_stated >= 10
    assert np.all(errs[:k_stated] <= 1e-4) and np.all(gaps[:k_stated] <= 1e-4)
    _beyond("tomo128 fp32 replay", K, k_stated, errs, R, sens)
    # Equal reconstruction error (the mixed-precision comparison: within 2 %
    # of FP64's) at the error minimum and at the stopping index.
    e64 = [rel(R.X[:, k], prob.x_true) for k in range(K)]
    e32 = [rel(G["X"][:, k], prob.x_true) for k in range(K)]
    kmin = int(np.argmin(e64))
    assert abs(e32[kmin] - e64[kmin]) <= 1e-4 * e64[kmin]
    assert abs(e32[R.k_stop - 1] - e64[R.k_stop - 1]) <= 2e-2 * e64[R.k_stop - 1]


def test_tomo128_fp64_free_full(lib, ctx, tomo):
    prob, R, sens, _ = tomo
    G = gpu_solve(lib, ctx, prob, "fp64", 100, "wgcv", grid=lambda_grid(),
                  grid_relative=True, bases=False)
    k_piv = pivot_prefix(R, TAU["fp64"], min(R.k_done, G["k_done"]))
    print(f"[tomo128 fp64 free] pivots well separated up to k = {k_piv}")
    assert k_piv >= 90
    assert list(G["piv_g"][:k_piv]) == R.piv_g[:k_piv]
    assert list(G["piv_t"][:k_piv]) == R.piv_t[:k_piv]
    # The bases never depend on lambda, so x_k is decided by the pivots up to
    # g(k) and by lambda_k alone.  The weighted GCV function of this problem
    # is flat at the small-lambda end (neighbouring grid values differ by
    # ~1e-10 relative), so lambda_k may be a near-tie: where the two sides
    # pick different grid points that must be one, and x_k is then not unique.
    tol = step_tolerances(sens[:k_piv], 2.0 ** -53, 1e-10)
    k_stated = int(np.argmax(tol > 1e-10)) if np.any(tol > 1e-10) else k_piv
    same, worst = 0, 0.0
    errs = np.full(k_piv, np.nan)
    for k in range(1, k_piv + 1):
        if G["lambda_idx"][k - 1] != R.lambda_idx[k - 1]:
            assert R.sep_lambda[k - 1] <= TAU["fp64"], k
            continue
        errs[k - 1] = rel(G["X"][:, k - 1], R.X[:, k - 1])
        if k <= k_stated:
            same += 1
            worst = max(worst, errs[k - 1])
            assert errs[k - 1] <= 1e-10, (k, errs[k - 1])
            check_ghat(G, R, k, "fp64")
    print(f"[tomo128 fp64 free] stated 1e-10 applies for k <= {k_stated}; x_k compared "
          f"there at {same} steps (same lambda), max err {worst:.2e}")
    _beyond("tomo128 fp64 free", k_piv, k_stated, errs, R, sens)
    assert same >= k_stated // 2


def test_tomo128_fp64_optimal_full(lib, ctx, tomo):
    """The optimal rule (eq. lambda) at full size.  The bases do not depend on
    lambda, so the oracle's wGCV run supplies L_k, H and beta; its optimal
    lambda_k and x_k follow from them with the oracle's own rule."""
    prob, R, _, runs = tomo
    grid = lambda_grid()
    G = gpu_solve(lib, ctx, prob, "fp64", 100, "optimal", grid=grid,
                  grid_relative=True, bases=False, x_true=prob.x_true)
    k_piv = pivot_prefix(R, TAU["fp64"], min(R.k_done, G["k_done"]))
    assert k_piv >= 90
    assert list(G["piv_g"][:k_piv]) == R.piv_g[:k_piv]
    assert list(G["piv_t"][:k_piv]) == R.piv_t[:k_piv]
    reg = RegParam("optimal", grid=grid, grid_relative=True, x_true=prob.x_true)
    x0 = np.zeros(prob.n)
    lams, idxs, seps = [], [], []
    Xo = np.zeros((prob.n, k_piv))
    for k in range(1, k_piv + 1):
        s, c, V = projected_svd(R.H[:k + 1, :k])
        lam, idx, sep, _ = select_lambda(reg, k, prob.m, R.beta, s, c, V, R.L[:, :k], x0)
        lams.append(lam)
        idxs.append(idx)
        seps.append(sep)
        Xo[:, k - 1] = R.L[:, :k] @ tikhonov_coeffs(R.beta, s, c, V, lam)
    # the sensitivity of these iterates, at the optimal lambda sequence
    sens = sensitivity_at(runs, lams, Xo, k_piv)
    tol = step_tolerances(sens, 2.0 ** -53, 1e-10)
    k_stated = int(np.argmax(tol > 1e-10)) if np.any(tol > 1e-10) else k_piv
    same, worst = 0, 0.0
    errs = np.full(k_piv, np.nan)
    for k in range(1, k_piv + 1):
        if G["lambda_idx"][k - 1] != idxs[k - 1]:
            assert seps[k - 1] <= TAU["fp64"], (k, idxs[k - 1], G["lambda_idx"][k - 1])
            continue
        errs[k - 1] = rel(G["X"][:, k - 1], Xo[:, k - 1])
        if k <= k_stated:
            same += 1
            worst = max(worst, errs[k - 1])
            assert errs[k - 1] <= 1e-10, (k, errs[k - 1])
    print(f"[tomo128 fp64 optimal] stated 1e-10 applies for k <= {k_stated}; lambda and "
          f"x_k compared there at {same} steps, max err {worst:.2e}")
    _beyond("tomo128 fp64 optimal", k_piv, k_stated, errs, R, sens)
    assert same >= k_stated // 2


def _psf_at(img_stack, P, pix, rows, cols, transpose):
    """(A v)(pix) or (A^T v)(pix) for every image in img_stack (count x rows x
    cols), from the definition: zero-boundary convolution / correlation."""
    ph, pw = P.shape
    ch, cw = ph // 2, pw // 2
    W = P if transpose else P[::-1, ::-1]  # correlation weights
    out = np.zeros((img_stack.shape[0], len(pix)))
    pad = np.pad(img_stack, ((0, 0), (ch, ch), (cw, cw)))
    for t, p in enumerate(pix):
        i, j = divmod(int(p), cols)
        patch = pad[:, i:i + ph, j:j + pw]
        out[:, t] = np.einsum("kab,ab->k", patch, W)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deblur1024_sampled(lib, ctx, prec):
    prob = config_problem("deblur1024")
    rows, cols = prob.image_shape
    K = 150
    grid = lambda_grid()
    G = gpu_solve(lib, ctx, prob, prec, K, "wgcv", grid=grid, grid_relative=True)
    assert G["status"] == lib.LSLU_OK and G["k_done"] == K
    L, D = G["L"], G["D"]
    # exact structure
    pg = [int(v) for v in G["piv_g"][:K]]
    pt = [int(v) for v in G["piv_t"][:K + 1]]
    assert len(set(pg)) == K and len(set(pt)) == K + 1
    for k in range(K):
        assert L[pg[k], k] == 1.0 and D[pt[k], k] == 1.0
        assert np.all(L[pg[:k], k] == 0.0) and np.all(D[pt[:k], k] == 0.0)
    assert np.abs(L).max() <= 1.0 and np.abs(D).max() <= 1.0
    # relations at sampled pixels: A L_k = D_{k+1} H, A^T D_k = L_k W_k
    rng = np.random.default_rng(5)
    pix = np.concatenate([rng.integers(0, prob.n, 48), pg[:8], [0, prob.n - 1]])
    H, W = G["H"][:K + 1, :K], G["W"][:K, :K]
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    AL = _psf_at(L.T.reshape(K, rows, cols), prob.psf, pix, rows, cols, False)
    DH = (D[pix, :K + 1] @ H).T
    mag = (np.abs(D[pix, :K + 1]) @ np.abs(H)).T + np.abs(AL)
    assert np.all(np.abs(AL - DH) <= 20 * K * u * (mag + 1e-300))
    ATD = _psf_at(D[:, :K].T.reshape(K, rows, cols), prob.psf, pix, rows, cols, True)
    LW = (L[pix, :K] @ W).T
    mag = (np.abs(L[pix, :K]) @ np.abs(W)).T + np.abs(ATD)
    assert np.all(np.abs(ATD - LW) <= 20 * K * u * (mag + 1e-300))
    # projected problem re-solved by the oracle from the library's H and beta
    reg = RegParam("wgcv", grid=grid, grid_relative=True)
    beta = G["beta"]
    worst_y = 0.0
    for k in (1, 2, 5, 20, 50, 100, 149, 150):
        s, c, V = projected_svd(H[:k + 1, :k])
        lam, li, sep, _ = select_lambda(reg, k, prob.m, beta, s, c, V, None, None)
        if sep > 1e-9:
            assert G["lambda_idx"][k - 1] == li, k
        y = tikhonov_coeffs(beta, s, c, V, G["lambda_k"][k - 1])
        worst_y = max(worst_y, rel(G["Y"][:k, k - 1], y))
        # x_k at sampled pixels from the library's own L and y_k
        xs = L[pix, :k] @ G["Y"][:k, k - 1]
        assert np.allclose(G["X"][pix, k - 1], xs, rtol=1e-5 if prec == "fp32" else 1e-12,
                           atol=1e-6 * np.abs(xs).max() if prec == "fp32" else 1e-14)
    print(f"[deblur1024 {prec}] max y_k error vs oracle projected solve {worst_y:.2e}")
    assert worst_y <= 1e-9
    e = rel(G["x"], prob.x_true)
    print(f"[deblur1024 {prec}] rel err vs x_true at k=150: {e:.4f}")
    # bit-identical repeat
    G2 = gpu_solve(lib, ctx, prob, prec, K, "wgcv", grid=grid, grid_relative=True,
                   bases=False)
    assert np.array_equal(G2["X"], G["X"]) and np.array_equal(G2["H"], G["H"])
