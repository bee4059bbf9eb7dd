"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rational arithmetic, the basis relations the paper proves (eq. nhr, eq. nhr2,
eq. h1), Krylov subspaces built by an orthogonal process, Algorithm 2 on the
normal equations, closed forms, brute-force minimisation of the projected
objectives (eq. quasi, eq. TP), the residual bounds of Theorems 1 and 2, the
trace forms of the GCV functions, and scaling/permutation symmetry.
"""

from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import RegParam, make_operator
from oracle.exact import hybrid_lslu_exact
from oracle.hessenberg import Status, hybrid_lslu, square_hessenberg_pivoted
from oracle.operators import DenseOp, PsfOp
from oracle.projected import (ghat_value, gcv_value, projected_svd,
                              tikhonov_coeffs, wgcv_value)
from workloads import (config_problem, lambda_grid, psf_deblur, random_dense,
                       tomography)

EPS = np.finfo(np.float64).eps


def _small_problems():
    return [
        random_dense(12, 9, seed=1, nu=0.05),
        random_dense(9, 12, seed=2, nu=0.05),
        random_dense(10, 10, seed=3, nu=0.05),
        tomography(16, 12, 23, 0.02, seed=5),
        psf_deblur(12, 3, 1.5, 0.01, seed=6),
    ]


# ---------------------------------------------------------------------------
# P2: exact structural invariants (unit lower triangular under the pivots)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", _small_problems(), ids=lambda p: p.name)
def test_basis_structure_exact(prob):
    op = make_operator(prob)
    K = min(8, prob.m, prob.n)
    r = hybrid_lslu(op, prob.b, K, RegParam("wgcv", grid=lambda_grid()))
    L, D = r.L, r.D
    # each basis vector: exactly 1 at its own pivot, exactly 0 at earlier ones
    for k, gk in enumerate(r.piv_g):
        assert L[gk, k] == 1.0
        for j in range(k):
            assert L[r.piv_g[j], k] == 0.0
    for k, tk in enumerate(r.piv_t):
        assert D[tk, k] == 1.0
        for j in range(k):
            assert D[r.piv_t[j], k] == 0.0
    assert np.all(np.abs(L) <= 1.0) and np.all(np.abs(D) <= 1.0)
    assert len(set(r.piv_g)) == len(r.piv_g)
    assert len(set(r.piv_t)) == len(r.piv_t)
    k = r.k_done
    assert np.all(np.tril(r.H[:k + 1, :k], -2) == 0)  # upper Hessenberg
    assert np.all(np.tril(r.W[:k, :k], -1) == 0)  # upper triangular
    # pivot values are the diagonal of W and the subdiagonal of H
    q1 = op.rmatvec(D[:, 0])
    assert r.W[0, 0] == q1[r.piv_g[0]]
    assert r.beta == prob.b[r.piv_t[0]]


# ---------------------------------------------------------------------------
# P3: the Hessenberg relations (eq. nhr, eq. nhr2, eq. h1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", _small_problems(), ids=lambda p: p.name)
def test_hessenberg_relations(prob):
    op = make_operator(prob)
    K = min(8, prob.m, prob.n)
    r = hybrid_lslu(op, prob.b, K)
    k = r.k_done
    L, D, H, W = r.L[:, :k], r.D[:, :k + 1], r.H[:k + 1, :k], r.W[:k, :k]
    AL = np.stack([op.matvec(L[:, j]) for j in range(k)], axis=1)
    ATD = np.stack([op.rmatvec(D[:, j]) for j in range(k)], axis=1)
    nA = np.linalg.norm(op.todense() if hasattr(op, "todense") else
                        np.stack([op.matvec(e) for e in np.eye(prob.n)], 1))
    tol = 10 * k * EPS
    # A L_k = D_{k+1} H_{k+1,k}
    assert np.linalg.norm(AL - D @ H) <= tol * nA * np.linalg.norm(L) * 10
    # A^T D_k = L_k W_k  (leading block of A^T D_{k+1} = L_{k+1} W_{k+1})
    assert np.linalg.norm(ATD - L @ W) <= tol * nA * np.linalg.norm(D) * 10
    # A^T A L_{k-1} = L_k W_k H_{k,k-1}
    if k >= 2:
        ATAL = np.stack([op.rmatvec(AL[:, j]) for j in range(k - 1)], axis=1)
        rhs = L @ W @ H[:k, :k - 1]
        assert (np.linalg.norm(ATAL - rhs)
                <= tol * nA * nA * np.linalg.norm(L) * 100)


# ---------------------------------------------------------------------------
# P4: the bases span the Krylov subspaces (eq. K1, eq. K2), checked against
# Golub-Kahan bidiagonalisation with full reorthogonalisation.
# ---------------------------------------------------------------------------

def _golub_kahan(A, b, k):
    m, n = A.shape
    U = np.zeros((m, k + 1))
    V = np.zeros((n, k))
    U[:, 0] = b / np.linalg.norm(b)
    for j in range(k):
        v = A.T @ U[:, j]
        for _ in range(2):
            v -= V[:, :j] @ (V[:, :j].T @ v)
        V[:, j] = v / np.linalg.norm(v)
        u = A @ V[:, j]
        for _ in range(2):
            u -= U[:, :j + 1] @ (U[:, :j + 1].T @ u)
        U[:, j + 1] = u / np.linalg.norm(u)
    return U, V


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_krylov_spans(seed):
    prob = random_dense(30, 20, seed=seed, nu=0.1)
    A = prob.A
    k = 6
    r = hybrid_lslu(DenseOp(A), prob.b, k)
    U, V = _golub_kahan(A, prob.b, k)
    ang_L = scipy.linalg.subspace_angles(r.L[:, :k], V)
    ang_D = scipy.linalg.subspace_angles(r.D[:, :k + 1], U)
    assert ang_L.max() < 1e-8
    assert ang_D.max() < 1e-8


# ---------------------------------------------------------------------------
# P5: equivalence with Algorithm 2 on the normal equations (eq. h1, eq. h2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [21, 22])
def test_equivalent_to_square_process_on_normal_equations(seed):
    prob = random_dense(14, 10, seed=seed, nu=0.1)
    A = prob.A
    k = 6
    r = hybrid_lslu(DenseOp(A), prob.b, k)
    # A^T A from v_0 = A^T r_0: same L, Hessenberg matrix W_{k+1} H_{k+1,k}
    Ls, Hs, p = square_hessenberg_pivoted(lambda v: A.T @ (A @ v),
                                          A.T @ prob.b, k - 1)
    assert p == r.piv_g[:len(p)]
    assert np.allclose(Ls, r.L[:, :Ls.shape[1]], rtol=0, atol=1e-10)
    WH = r.W[:k, :k] @ r.H[:k, :k - 1]
    assert np.allclose(Hs, WH[:Hs.shape[0], :Hs.shape[1]], rtol=1e-9,
                       atol=1e-10 * np.abs(WH).max())
    # A A^T from r_0: same D, Hessenberg matrix H_{k+1,k} W_k (eq. h2)
    Ds, Hs2, p2 = square_hessenberg_pivoted(lambda v: A @ (A.T @ v),
                                            prob.b, k - 1)
    assert p2 == r.piv_t[:len(p2)]
    assert np.allclose(Ds, r.D[:, :Ds.shape[1]], rtol=0, atol=1e-10)
    HW = r.H[:k, :k - 1] @ r.W[:k - 1, :k - 1]
    assert np.allclose(Hs2, HW[:Hs2.shape[0], :Hs2.shape[1]], rtol=1e-9,
                       atol=1e-10 * np.abs(HW).max())


# ---------------------------------------------------------------------------
# P1: exact rational arithmetic on tiny integer problems
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,seed", [((5, 4), 31), ((4, 6), 32),
                                        ((6, 6), 33), ((7, 5), 34)])
def test_fp64_matches_exact_rationals(shape, seed):
    prob = random_dense(*shape, seed=seed, integer=True)
    K = min(shape)
    ex = hybrid_lslu_exact(prob.A.astype(int).tolist(),
                           prob.b.astype(int).tolist(), K)
    r = hybrid_lslu(DenseOp(prob.A), prob.b, K)
    kd = min(ex["k_done"], r.k_done)
    assert kd >= 1
    assert r.piv_t[:kd] == ex["piv_t"][:kd]
    assert r.piv_g[:kd] == ex["piv_g"][:kd]
    for k in range(kd):
        xe = np.array([float(v) for v in ex["X"][k]])
        assert np.linalg.norm(r.X[:, k] - xe) <= 1e-10 * max(1.0, np.linalg.norm(xe))
        le = np.array([float(v) for v in ex["L"][k]])
        assert np.allclose(r.L[:, k], le, rtol=0, atol=1e-12)


def test_pivot_tie_goes_to_smallest_index():
    # |b| has its maximum 5 at rows 1 and 3; the pivot must be row 1.
    A = np.eye(4) + 0.25 * np.diag(np.ones(3), 1)
    b = np.array([1.0, -5.0, 2.0, 5.0])
    r = hybrid_lslu(DenseOp(A), b, 2)
    assert r.piv_t[0] == 1
    assert r.beta == -5.0
    ex = hybrid_lslu_exact([[Fraction(v) for v in row] for row in A],
                           [Fraction(v) for v in b], 2)
    assert ex["piv_t"][0] == 1
    # a tie among non-pivot q entries: A = I, b with two equal maxima
    r2 = hybrid_lslu(DenseOp(np.eye(3)), np.array([2.0, 0.0, -2.0]), 1)
    assert r2.piv_t[0] == 0 and r2.piv_g[0] == 0


def test_rank_deficient_breaks_down_on_q_side_in_rationals():
    rng = np.random.default_rng(41)
    B = rng.integers(-3, 4, size=(6, 2))
    C = rng.integers(-3, 4, size=(2, 5))
    A = (B @ C).tolist()  # rank 2
    b = rng.integers(-3, 4, size=6).tolist()
    ex = hybrid_lslu_exact(A, b, 5)
    assert ex["status"] == Status.BREAKDOWN_Q
    assert ex["k_done"] == 2  # l_3 cannot be formed


# ---------------------------------------------------------------------------
# P7: consistent square full-rank system is solved at full dimension
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(3, 51), (5, 52), (6, 53), (8, 54)])
def test_square_consistent_system_solved_exactly(n, seed):
    rng = np.random.default_rng(seed)
    while True:
        A = rng.integers(-3, 4, size=(n, n)).astype(float) + 4 * np.eye(n)
        if np.linalg.cond(A) < 100:
            break
    x_true = rng.integers(-3, 4, size=n).astype(float)
    b = A @ x_true
    r = hybrid_lslu(DenseOp(A), b, n)
    assert r.status == Status.BREAKDOWN_U and r.k_done == n
    assert np.linalg.norm(r.x - x_true) <= 1e-12 * np.linalg.norm(x_true) * 10
    ex = hybrid_lslu_exact(A.astype(int).tolist(), b.astype(int).tolist(), n)
    assert ex["status"] == Status.BREAKDOWN_U and ex["k_done"] == n
    assert [Fraction(int(v)) for v in x_true] == ex["x"]


# ---------------------------------------------------------------------------
# P6: closed forms and degenerate inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("c,lam", [(2.0, 0.0), (0.5, 0.3), (-3.0, 1.0)])
def test_scaled_identity_closed_form(c, lam):
    rng = np.random.default_rng(61)
    b = rng.standard_normal(7)
    reg = RegParam("fixed", lam=lam) if lam else RegParam("none")
    r = hybrid_lslu(DenseOp(c * np.eye(7)), b, 5, reg)
    assert r.status == Status.BREAKDOWN_U and r.k_done == 1
    assert np.allclose(r.x, c * b / (c * c + lam * lam), rtol=4 * EPS, atol=0)


def test_zero_rhs():
    r = hybrid_lslu(DenseOp(np.eye(3)), np.zeros(3), 2)
    assert r.status == Status.ZERO_RHS and r.k_done == 0
    assert np.all(r.x == 0)


def test_rhs_in_adjoint_nullspace_breaks_down_on_q_side():
    A = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    r = hybrid_lslu(DenseOp(A), np.array([0.0, 0.0, 3.0]), 2)
    assert r.status == Status.BREAKDOWN_Q and r.k_done == 0
    assert np.all(r.x == 0)


# ---------------------------------------------------------------------------
# P8: the iterate minimises the projected objective (eq. quasi and eq. TP),
# computed by brute force from the stored bases -- independent of H and SVD.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["none", "fixed", "wgcv"])
@pytest.mark.parametrize("prob", _small_problems()[:4], ids=lambda p: p.name)
def test_iterate_minimises_projected_objective(prob, kind):
    op = make_operator(prob)
    K = min(7, prob.m, prob.n)
    reg = RegParam(kind, lam=0.05, grid=lambda_grid(), grid_relative=True)
    r = hybrid_lslu(op, prob.b, K, reg)
    for k in range(1, r.k_done + 1):
        L = r.L[:, :k]
        Dp = np.linalg.pinv(r.D[:, :k + 1])
        AL = np.stack([op.matvec(L[:, j]) for j in range(k)], axis=1)
        lam = r.lambdas[k - 1]
        M = np.vstack([Dp @ AL, lam * np.eye(k)])
        rhs = np.concatenate([Dp @ prob.b, np.zeros(k)])
        y, *_ = np.linalg.lstsq(M, rhs, rcond=None)
        xb = L @ y
        kap = np.linalg.cond(M)
        assert (np.linalg.norm(r.X[:, k - 1] - xb)
                <= 1e-12 * kap * np.linalg.norm(xb) + 1e-14)


# ---------------------------------------------------------------------------
# P9: Theorem 1 and Theorem 2 residual bounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", _small_problems()[:4], ids=lambda p: p.name)
def test_residual_bounds_theorems(prob):
    op = make_operator(prob)
    K = min(7, prob.m, prob.n)
    lam = 0.05
    r_lu = hybrid_lslu(op, prob.b, K)
    r_h = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam))
    b = prob.b
    for k in range(1, min(r_lu.k_done, r_h.k_done) + 1):
        L = r_lu.L[:, :k]
        AL = np.stack([op.matvec(L[:, j]) for j in range(k)], axis=1)
        # LSQR's iterate minimises ||b - A x|| over range(L_k) (Theorem 1)
        y, *_ = np.linalg.lstsq(AL, b, rcond=None)
        r_qr = np.linalg.norm(b - AL @ y)
        r_lu_k = np.linalg.norm(b - op.matvec(r_lu.X[:, k - 1]))
        kap = np.linalg.cond(r_lu.D[:, :k + 1])
        assert r_qr <= r_lu_k * (1 + 1e-12)
        assert r_lu_k <= kap * r_qr * (1 + 1e-12)
        # Theorem 2, hybrid residual hr(x) = [b; 0] - [A; lam I] x
        M = np.vstack([AL, lam * L])
        rhs = np.concatenate([b, np.zeros(prob.n)])
        yh, *_ = np.linalg.lstsq(M, rhs, rcond=None)
        hr_qr = np.linalg.norm(rhs - M @ yh)
        xh = r_h.X[:, k - 1]
        hr_lu = np.linalg.norm(np.concatenate([b - op.matvec(xh), -lam * xh]))
        Dbar = scipy.linalg.block_diag(r_h.D[:, :k + 1], r_h.L[:, :k])
        kbar = np.linalg.cond(Dbar)
        assert hr_qr <= hr_lu * (1 + 1e-12)
        assert hr_lu <= kbar * hr_qr * (1 + 1e-12)


# ---------------------------------------------------------------------------
# P10: GCV, weighted GCV and Ghat -- SVD forms against their defining trace /
# residual forms with explicit matrices (eq. gcv1, eq. wgcv_projected1,
# eq. stop1).
# ---------------------------------------------------------------------------

def _explicit_Hlam(H, lam):
    k = H.shape[1]
    return np.linalg.solve(H.T @ H + lam * lam * np.eye(k), H.T)


@pytest.mark.parametrize("seed", [71, 72, 73])
def test_gcv_forms(seed):
    rng = np.random.default_rng(seed)
    k = 6
    H = np.triu(rng.standard_normal((k + 1, k)), -1)
    beta = 1.7
    e1 = np.zeros(k + 1)
    e1[0] = 1.0
    s, c, V = projected_svd(H)
    for lam in [1e-3, 0.1, 2.0]:
        Hl = _explicit_Hlam(H, lam)
        P = H @ Hl
        res = np.linalg.norm((np.eye(k + 1) - P) @ (beta * e1)) ** 2
        g_tr = k * res / np.trace(np.eye(k + 1) - P) ** 2
        assert np.isclose(gcv_value(k, beta, s, c, lam), g_tr, rtol=1e-11)
        for om in [0.1, 0.5, 1.0]:
            w_tr = k * res / np.trace(np.eye(k + 1) - om * P) ** 2
            assert np.isclose(wgcv_value(k, beta, s, c, lam, om), w_tr,
                              rtol=1e-11)
        # Tikhonov coefficients against the normal-equations solution (eq. 2)
        y = tikhonov_coeffs(beta, s, c, V, lam)
        assert np.allclose(y, Hl @ (beta * e1), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("prob", _small_problems()[:3], ids=lambda p: p.name)
def test_ghat_trace_form(prob):
    """Ghat(k) = n ||D^+ (I - A A_k^+) b||^2 / trace(I - A A_k^+)^2 with
    A_k^+ = L_k H_lambda^+ D^+_{k+1} (eq. stop1, x_0 = 0)."""
    op = make_operator(prob)
    A = op.todense()
    K = min(6, prob.m, prob.n)
    r = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=0.07))
    for k in range(1, r.k_done + 1):
        Dp = np.linalg.pinv(r.D[:, :k + 1])
        H = r.H[:k + 1, :k]
        Ak = r.L[:, :k] @ _explicit_Hlam(H, 0.07) @ Dp
        Mres = np.eye(prob.m) - A @ Ak
        num = prob.n * np.linalg.norm(Dp @ Mres @ prob.b) ** 2
        den = np.trace(Mres) ** 2
        assert np.isclose(r.ghat[k - 1], num / den, rtol=1e-9)


# ---------------------------------------------------------------------------
# P11: scaling and permutation symmetry of the method
# ---------------------------------------------------------------------------

def test_power_of_two_scaling_is_exact():
    prob = random_dense(15, 11, seed=81, nu=0.1)
    A, b = prob.A, prob.b
    K = 7
    reg = RegParam("wgcv", grid=lambda_grid(), grid_relative=True)
    r = hybrid_lslu(DenseOp(A), b, K, reg)
    rb = hybrid_lslu(DenseOp(A), 8.0 * b, K, reg)
    assert rb.piv_t == r.piv_t and rb.piv_g == r.piv_g
    assert np.array_equal(rb.L, r.L) and np.array_equal(rb.D, r.D)
    assert np.array_equal(rb.lambda_idx, r.lambda_idx)
    assert np.allclose(rb.X, 8.0 * r.X, rtol=1e-13, atol=0)
    ra = hybrid_lslu(DenseOp(0.25 * A), b, K, reg)
    assert ra.piv_t == r.piv_t and ra.piv_g == r.piv_g
    assert np.array_equal(ra.L, r.L) and np.array_equal(ra.D, r.D)
    assert np.array_equal(ra.H, 0.25 * r.H)
    assert np.array_equal(ra.lambda_idx, r.lambda_idx)
    assert np.allclose(ra.X, 4.0 * r.X, rtol=1e-12, atol=0)


def test_row_and_column_permutation():
    prob = random_dense(13, 9, seed=82, nu=0.1)
    rng = np.random.default_rng(83)
    pr = rng.permutation(13)
    pc = rng.permutation(9)
    K = 6
    r = hybrid_lslu(DenseOp(prob.A), prob.b, K)
    Ap = prob.A[pr][:, pc]
    rp = hybrid_lslu(DenseOp(Ap), prob.b[pr], K)
    inv_r = np.argsort(pr)
    inv_c = np.argsort(pc)
    assert [int(inv_r[i]) for i in r.piv_t] == rp.piv_t
    assert [int(inv_c[i]) for i in r.piv_g] == rp.piv_g
    assert np.allclose(rp.x, r.x[pc], rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# P12: the optimal lambda is the grid point with the smallest error
# ---------------------------------------------------------------------------

def test_optimal_lambda_brute_force():
    prob = config_problem("dense256")
    op = make_operator(prob)
    grid = lambda_grid()
    r = hybrid_lslu(op, prob.b, 12, RegParam("optimal", grid=grid,
                                             x_true=prob.x_true))
    for k in range(1, r.k_done + 1):
        H = r.H[:k + 1, :k]
        errs = []
        for lam in grid:
            M = np.vstack([H, lam * np.eye(k)])
            rhs = np.zeros(2 * k + 1)
            rhs[0] = r.beta
            y, *_ = np.linalg.lstsq(M, rhs, rcond=None)
            errs.append(np.linalg.norm(r.L[:, :k] @ y - prob.x_true))
        errs = np.array(errs)
        best = int(np.argmin(errs))
        srt = np.sort(errs)
        if (srt[1] - srt[0]) / srt[0] > 1e-8:
            assert r.lambda_idx[k - 1] == best


# ---------------------------------------------------------------------------
# Operators: the PSF convolution/correlation and the CSR matrix, against
# matrices built entry by entry from their definitions.
# ---------------------------------------------------------------------------

def test_psf_operator_definition():
    rng = np.random.default_rng(91)
    rows, cols, ph, pw = 7, 9, 5, 3
    P = rng.standard_normal((ph, pw))  # deliberately not symmetric
    op = PsfOp(P, (rows, cols))
    n = rows * cols
    A = np.zeros((n, n))
    for i in range(rows):
        for j in range(cols):
            for a in range(ph):
                for bb in range(pw):
                    si, sj = i - a + ph // 2, j - bb + pw // 2
                    if 0 <= si < rows and 0 <= sj < cols:
                        A[i * cols + j, si * cols + sj] += P[a, bb]
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    assert np.allclose(op.matvec(x), A @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(op.rmatvec(y), A.T @ y, rtol=1e-13, atol=1e-13)


def test_csr_operator_and_generator_shapes():
    prob = tomography(16, 12, 23, 0.02, seed=5)
    op = make_operator(prob)
    A = np.zeros((prob.m, prob.n))
    for r in range(prob.m):
        for p in range(prob.indptr[r], prob.indptr[r + 1]):
            A[r, prob.indices[p]] += prob.data[p]
    x = np.random.default_rng(0).standard_normal(prob.n)
    y = np.random.default_rng(1).standard_normal(prob.m)
    assert np.allclose(op.matvec(x), A @ x, rtol=1e-13, atol=1e-12)
    assert np.allclose(op.rmatvec(y), A.T @ y, rtol=1e-13, atol=1e-12)
    # sorted, in range, no explicit zeros
    for r in range(prob.m):
        cols = prob.indices[prob.indptr[r]:prob.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
    assert np.all(prob.data != 0)
    # noise level is the paper's definition ||e|| / ||A x_true||
    Ax = A @ prob.x_true
    assert np.isclose(np.linalg.norm(prob.b - Ax) / np.linalg.norm(Ax), 0.02,
                      rtol=1e-10)


def test_lambda_grid_tie_smallest_index():
    from oracle.projected import _grid_argmin
    idx, sep = _grid_argmin([3.0, 1.0, 1.0, 2.0])
    assert idx == 1 and sep == 0.0


def test_pivot_search_separation_and_stop_rule():
    from oracle.hessenberg import pivot_search
    v = np.array([0.5, -4.0, 3.0, 4.0, 1.0])
    pos, amax, sep = pivot_search(v, np.arange(5), 0)
    assert pos == 1 and amax == 4.0 and sep == 0.0  # tie 4 / -4
    pos, amax, sep = pivot_search(v, np.array([1, 0, 2, 4, 3]), 1)
    assert pos == 4 and amax == 4.0 and sep == 0.25  # candidates 0.5, 3, 1, 4
    prob = config_problem("dense256")
    op = make_operator(prob)
    reg = RegParam("wgcv", grid=lambda_grid())
    r = hybrid_lslu(op, prob.b, 20, reg, stop_tol=1e-2)
    g = r.ghat
    ks = [k for k in range(1, len(g)) if abs(g[k] - g[k - 1]) / g[0] < 1e-2]
    assert r.k_stop == ks[0]
    re = hybrid_lslu(op, prob.b, 20, reg, stop_tol=1e-2, early_stop=True)
    assert re.k_stop == r.k_stop
    assert np.array_equal(re.x, r.X[:, r.k_stop - 1])


# ---------------------------------------------------------------------------
# Sampled pivots (the variant of Section 2.2 / Fig. 1, reading R19)
# ---------------------------------------------------------------------------

def _sampled_winner(vec, rows, earlier, s):
    """Brute force: the largest |vec| among the first s listed rows that are
    not earlier pivots, ties to the smallest row; None if that is 0."""
    sample = [int(r) for r in rows if r >= 0 and int(r) not in earlier][:s]
    if not sample or max(abs(vec[r]) for r in sample) == 0.0:
        return None
    return max(sample, key=lambda r: (abs(vec[r]), -r))


@pytest.mark.parametrize("seed,s", [(1, 3), (2, 5), (3, 12)])
def test_sampled_pivot_rule_by_brute_force(seed, s):
    from workloads import pivot_sample_lists
    prob = random_dense(40, 28, seed=seed, nu=0.05)
    op = make_operator(prob)
    K = 10
    lists = pivot_sample_lists(prob.m, prob.n, K, s, seed=seed)
    r = hybrid_lslu(op, prob.b, K, pivot_sample=(lists, s))
    # every search's winner, re-derived from the result's own vectors: q_k is
    # a multiple of l_k, u_k of d_{k+1}, r_0 of d_1 (pivot entries exactly 1)
    assert r.piv_t[0] == _sampled_winner(r.D[:, 0], lists[0], set(), s)
    for k in range(1, r.k_done + 1):
        wg = _sampled_winner(r.L[:, k - 1], lists[2 * k - 1], set(r.piv_g[:k - 1]), s)
        assert wg is not None and r.piv_g[k - 1] == wg
        if k < len(r.piv_t):
            wt = _sampled_winner(r.D[:, k], lists[2 * k], set(r.piv_t[:k]), s)
            assert wt is not None and r.piv_t[k] == wt
    # any pivot choice keeps the Hessenberg relations of Section 2.2
    k = r.k_done
    A = prob.A
    assert np.allclose(A @ r.L[:, :k], r.D[:, :k + 1] @ r.H[:k + 1, :k], atol=1e-10)
    assert np.allclose(A.T @ r.D[:, :k], r.L[:, :k] @ r.W[:k, :k], atol=1e-10)


def test_sampled_pivots_with_every_row_listed_equal_full_pivoting():
    prob = random_dense(36, 25, seed=4, nu=0.05)
    op = make_operator(prob)
    K = 12
    rng = np.random.default_rng(7)
    L = K + max(prob.m, prob.n)
    lists = np.full((2 * K + 1, L), -1, dtype=np.int32)
    for i in range(2 * K + 1):
        length = prob.m if i % 2 == 0 else prob.n
        lists[i, :length] = rng.permutation(length)
    reg = RegParam("wgcv", grid=lambda_grid(), grid_relative=True)
    full = hybrid_lslu(op, prob.b, K, reg)
    samp = hybrid_lslu(op, prob.b, K, reg, pivot_sample=(lists, L))
    assert samp.piv_t == full.piv_t and samp.piv_g == full.piv_g
    assert np.array_equal(samp.X, full.X)


def test_sampled_pivot_falls_back_to_full_search_on_a_zero_sample():
    prob = random_dense(30, 20, seed=5, nu=0.05)
    op = make_operator(prob)
    K, s = 4, 3
    lists = np.full((2 * K + 1, s + K), -1, dtype=np.int32)
    for i in range(2 * K + 1):
        lists[i, :s + K] = np.arange(s + K)
    b = prob.b.copy()
    b[:s + K] = 0.0  # every listed row of r_0 is zero
    r = hybrid_lslu(op, b, K, pivot_sample=(lists, s))
    full_t1 = int(np.argmax(np.abs(b)))
    assert r.piv_t[0] == full_t1 and abs(r.beta) == np.abs(b).max()


# ---------------------------------------------------------------------------
# d loss / d lambda of the projected Tikhonov solve (eq. TSP, eq. lambda)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lam", [1e-3, 0.02, 0.3])
def test_dloss_dlambda_against_central_differences(lam):
    from oracle.projected import dloss_dlambda, tikhonov_coeffs_dlambda
    prob = config_problem("dense256")
    op = make_operator(prob)
    r = hybrid_lslu(op, prob.b, 15)
    x0 = np.zeros(prob.n)
    for k in (3, 8, 15):
        s, c, V = projected_svd(r.H[:k + 1, :k])
        Lk = r.L[:, :k]

        def loss(l):
            y = tikhonov_coeffs(r.beta, s, c, V, l)
            return float(np.sum((x0 + Lk @ y - prob.x_true) ** 2))

        h = lam * 1e-4
        fd = (loss(lam + h) - loss(lam - h)) / (2 * h)
        g = dloss_dlambda(r.beta, s, c, V, lam, Lk, x0, prob.x_true)
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (k, g, fd)
        # dy/dlambda also from the normal equations, without the SVD
        Hk = r.H[:k + 1, :k]
        y = tikhonov_coeffs(r.beta, s, c, V, lam)
        dy = -2 * lam * np.linalg.solve(Hk.T @ Hk + lam * lam * np.eye(k), y)
        assert np.allclose(tikhonov_coeffs_dlambda(r.beta, s, c, V, lam), dy,
                           rtol=1e-7, atol=1e-9 * np.abs(dy).max())


# ---------------------------------------------------------------------------
# The lambda choice itself: grid index and value of the GCV and weighted-GCV
# rules, by brute force from the trace forms
# ---------------------------------------------------------------------------

def _trace_form_index(H, beta, k, omega, grid):
    """Index of the smallest G(omega, lambda) over the grid (ties: smallest
    index), with G the weighted GCV function of the projected problem in its
    trace form (eq. wgcv_projected1; omega = 1 is eq. gcv1):
        k ||(I - H H_lam^+) beta e_1||^2 / trace(I - omega H H_lam^+)^2,
    H_lam^+ = (H^T H + lam^2 I)^-1 H^T formed explicitly."""
    e1 = np.zeros(k + 1)
    e1[0] = beta
    vals = []
    for lam in grid:
        P = H @ np.linalg.solve(H.T @ H + lam * lam * np.eye(k), H.T)
        res = np.linalg.norm(e1 - P @ e1) ** 2
        vals.append(k * res / np.trace(np.eye(k + 1) - omega * P) ** 2)
    vals = np.array(vals)
    return int(np.flatnonzero(vals == vals.min())[0])


@pytest.mark.parametrize("rule", ["wgcv", "gcv"])
@pytest.mark.parametrize("prob,K", [(None, 30), ("tomo", 25)], ids=["blur48", "tomo16"])
def test_lambda_choice_by_brute_force(rule, prob, K):
    """At every k the oracle's lambda_k is sigma_1(H_{k+1,k}) times the grid
    value minimising the trace form with omega = (k+1)/m for weighted GCV (the
    weight the end of Section 3.2.1 adopts) and omega = 1 for GCV; sigma_1
    from numpy's singular values of the stored H.  On the 48-row problem
    (omega from 2/48 to 31/48) omega = k/m or (k+2)/m, or a grid scaled by
    sigma_k, picks a different lambda at some k, so an off-by-one weight or
    the wrong scale does not pass."""
    from workloads import dense_blur_1d
    prob = (dense_blur_1d(48, 2.0, 0.05, seed=3) if prob is None
            else tomography(16, 12, 23, 0.02, seed=5))
    grid = lambda_grid(120)
    r = hybrid_lslu(make_operator(prob), prob.b, K,
                    RegParam(rule, grid=grid, grid_relative=True))
    assert r.k_done == K
    m = prob.m
    shifted = {0: 0, 2: 0, "smin": 0}
    for k in range(1, K + 1):
        H = r.H[:k + 1, :k]
        sv = np.linalg.svd(H, compute_uv=False)
        omega = (k + 1) / m if rule == "wgcv" else 1.0
        idx = _trace_form_index(H, r.beta, k, omega, sv[0] * grid)
        assert r.lambda_idx[k - 1] == idx, (k, r.lambda_idx[k - 1], idx)
        assert np.isclose(r.lambdas[k - 1], sv[0] * grid[idx], rtol=1e-13, atol=0)
        if rule == "wgcv" and m == 48:
            for d in (0, 2):
                shifted[d] += _trace_form_index(H, r.beta, k, (k + d) / m, sv[0] * grid) != idx
            shifted["smin"] += _trace_form_index(H, r.beta, k, omega, sv[-1] * grid) != idx
    if rule == "wgcv" and m == 48:
        assert all(v > 0 for v in shifted.values()), shifted
