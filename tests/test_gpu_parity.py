"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Protocol:
* free mode -- the library picks its own pivots and lambda; pivots and x_k
  must match the oracle as long as every pivot/lambda search that decides x_k
  is well separated in the oracle (separation above tau);
* replay mode -- the library follows the oracle's pivots and lambda indices
  and x_k, H and W must match at every k.
Tolerances on ||x_k - x_oracle||/||x_oracle|| and on the relative residual gap:
1e-10 in FP64, 1e-4 in FP32.  BF16OP runs report their error against x_true.
"""

import numpy as np
import pytest

from gpu_helpers import (TAU, TOL, check_basis_invariants, check_ghat,
                         check_relations, gpu_solve, pivot_prefix, rel,
                         replay_from, residual_gap, well_separated_prefix)
from oracle import RegParam, make_operator
from oracle.hessenberg import Status, hybrid_lslu
from workloads import (config_problem, lambda_grid, psf_deblur, random_dense,
                       tomography)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.lslu_create(0)
    yield c
    lib.lslu_destroy(c)


def _reg(kind, relative, lam=0.05, x_true=None):
    return RegParam(kind, lam=lam, grid=lambda_grid(), grid_relative=relative,
                    x_true=x_true)


def _compare(lib, ctx, prob, prec, K, kind, relative, lam=0.05, replay=True,
             check_free=True, kappa_cap=None, pivot_sample=None):
    """Run oracle + GPU (free and replay) and check the parity bar."""
    op = make_operator(prob)
    xt = prob.x_true if kind == "optimal" else None
    R = hybrid_lslu(op, prob.b, K, _reg(kind, relative, lam, x_true=xt),
                    pivot_sample=pivot_sample)
    grid = lambda_grid() if kind in ("wgcv", "gcv", "optimal") else None
    tol = TOL[prec]
    if check_free:
        G = gpu_solve(lib, ctx, prob, prec, K, kind, lam, grid, relative, x_true=xt,
                      pivot_sample=pivot_sample)
        # a sampled pivot is the largest entry of its sample only, so the
        # entries of the bases are not bounded by 1 then
        check_basis_invariants(G, prob.m, prob.n,
                               bound=1.0 if pivot_sample is None else np.inf)
        k_piv = pivot_prefix(R, TAU[prec], min(R.k_done, G["k_done"]))
        assert list(G["piv_g"][:k_piv]) == R.piv_g[:k_piv]
        assert list(G["piv_t"][:k_piv]) == R.piv_t[:k_piv]
        k_ok = well_separated_prefix(R, TAU[prec], min(R.k_done, G["k_done"]))
        if prec == "fp64":
            for k in range(1, k_ok + 1):
                if kappa_cap and G["sigma_max"][k - 1] / G["sigma_min"][k - 1] > kappa_cap:
                    break
                assert rel(G["X"][:, k - 1], R.X[:, k - 1]) <= tol, k
                assert G["lambda_idx"][k - 1] == R.lambda_idx[k - 1] or R.lambda_idx[k - 1] < 0
                check_ghat(G, R, k, prec)
    if replay:
        Kr = min(K, R.k_done)
        ps = None
        if pivot_sample is not None:  # the lists of a Kr-iteration solve
            rows, ssz = pivot_sample
            ps = (rows[:2 * Kr + 1], ssz)
        G = gpu_solve(lib, ctx, prob, prec, Kr, kind, lam, grid, relative,
                      replay=replay_from(R, Kr), x_true=xt, pivot_sample=ps)
        check_basis_invariants(G, prob.m, prob.n,
                               bound=1.0 + 10 * TAU[prec] if pivot_sample is None else np.inf)
        assert G["k_done"] == Kr
        worst = []
        for k in range(1, Kr + 1):
            kap = G["sigma_max"][k - 1] / G["sigma_min"][k - 1]
            e = rel(G["X"][:, k - 1], R.X[:, k - 1])
            g = residual_gap(op, prob.b, G["X"][:, k - 1], R.X[:, k - 1])
            worst.append((k, e, g, kap))
            if kappa_cap is None or kap <= kappa_cap:
                assert e <= tol and g <= tol, (k, e, g, kap)
                check_ghat(G, R, k, prec)
        print(f"[{prob.name} {prec} {kind}] max x err "
              f"{max(w[1] for w in worst):.3e} max residual gap "
              f"{max(w[2] for w in worst):.3e}")
        # The GPU's own H, W, L, D satisfy the Hessenberg relations to the
        # rounding of its working precision; H and W also match the oracle's
        # entry by entry (relative to their largest entry), in FP64 over the
        # whole solve and in FP32 over the steps whose iterates were held to
        # the stated tolerance above (the kappa cap)
        check_relations(G, op, prec)
        kd = G["k_done"]
        if prec == "fp32" and kappa_cap is not None:
            for k in range(1, kd + 1):
                if G["sigma_max"][k - 1] / G["sigma_min"][k - 1] > kappa_cap:
                    kd = k - 1
                    break
        if prec in ("fp64", "fp32") and kd > 0:
            Hs = np.abs(R.H[:kd + 1, :kd]).max()
            Ws = np.abs(R.W[:kd, :kd]).max()
            dH = np.abs(G["H"][:kd + 1, :kd] - R.H[:kd + 1, :kd]).max()
            dW = np.abs(G["W"][:kd, :kd] - R.W[:kd, :kd]).max()
            print(f"[{prob.name} {prec} {kind}] H, W against the oracle over k <= {kd}: "
                  f"{dH / Hs:.2e}, {dW / Ws:.2e} of their largest entries")
            assert dH <= tol * 10 * Hs and dW <= tol * 10 * Ws
        return R, G
    return R, None


# --------------------------------------------------------------- operators

def _bound(Aabs_x, prec, nterms):
    u = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16op": 2.0 ** -8, "fp16op": 2.0 ** -11,
         "fp8op": 2.0 ** -4}[prec]
    acc = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -53, "bf16op": 2.0 ** -24, "fp16op": 2.0 ** -24,
           "fp8op": 2.0 ** -24}[prec]
    return (4 * u + nterms * acc) * Aabs_x + 1e-300


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16op", "fp16op", "fp8op"])
@pytest.mark.parametrize("which", ["dense", "dense96x64", "dense90x64", "csr", "psf31",
                                   "psf_nonsym", "psf_rand31", "psf_rand9x31", "psf_rand31x3"])
def test_operator_products(lib, ctx, which, prec):
    """Every product within (4u + n_terms u_sum)|A||x| of the FP64 product.
    The dense 96 x 64 and 90 x 64 shapes take the matrix-core dense product
    of the 16- and 8-bit modes (row lengths multiples of 16 and 32).
    The random full-width PSFs (all 31 columns, or rows, carry weights of
    order one) pin every diagonal of the banded form the 16- and 8-bit modes
    compute the PSF product in; the image widths (77, 70, 130) are not
    multiples of the 64-column tile and two are not multiples of 4."""
    import torch
    rng = np.random.default_rng(7)
    if which == "dense":
        prob = random_dense(37, 53, seed=3)
    elif which == "dense96x64":  # 16- and 8-bit modes: matrix cores both ways
        prob = random_dense(96, 64, seed=31)
    elif which == "dense90x64":  # A on the matrix cores (ragged row group), A^T not
        prob = random_dense(90, 64, seed=32)
    elif which == "csr":
        prob = tomography(20, 15, 29, 0.02, seed=4)
    elif which == "psf31":
        prob = psf_deblur(45, 15, 2.5, 0.01, seed=5, cols=77)
    elif which == "psf_nonsym":
        prob = psf_deblur(33, 2, 1.0, 0.01, seed=6, cols=70)
        prob.psf = rng.standard_normal((5, 3))
    else:
        shape = {"psf_rand31": (31, 31), "psf_rand9x31": (9, 31), "psf_rand31x3": (31, 3)}[which]
        prob = psf_deblur(50, 2, 1.0, 0.01, seed=8, cols=130 if shape[1] == 31 else 77)
        prob.psf = rng.uniform(0.25, 1.0, shape) * rng.choice([-1.0, 1.0], shape)
    op_or = make_operator(prob)
    absop = type(op_or)
    dt = torch.float64 if prec == "fp64" else torch.float32
    op = lib.make_operator(ctx, prob, lib.PRECISIONS[prec])
    try:
        for tr in (0, 1):
            nin, nout = (prob.n, prob.m) if tr == 0 else (prob.m, prob.n)
            x = rng.standard_normal(nin)
            if prec != "fp64":
                x = x.astype(np.float32).astype(np.float64)
            xt = torch.tensor(x, dtype=dt, device="cuda")
            yt = torch.full((nout,), np.nan, dtype=dt, device="cuda")
            lib.lslu_op_apply(ctx, op, tr, xt, yt)
            torch.cuda.synchronize()
            y = yt.double().cpu().numpy()
            ref = op_or.rmatvec(x) if tr else op_or.matvec(x)
            # |A| |x| via the oracle operator on absolute values
            if prob.kind == "dense":
                aop = absop(np.abs(prob.A))
            elif prob.kind == "csr":
                aop = absop(prob.m, prob.n, prob.indptr, prob.indices, np.abs(prob.data))
            else:
                aop = absop(np.abs(prob.psf), prob.image_shape)
            mag = aop.rmatvec(np.abs(x)) if tr else aop.matvec(np.abs(x))
            nterms = 600
            bound = _bound(mag, prec, nterms)
            if prec == "fp8op":
                # E4M3's smallest spacing is 2^-9: an entry of A or x below
                # 2^-6 rounds with an absolute error up to 2^-10, not a
                # relative one (short ray segments flush to zero), so each
                # term adds 2^-10 (|x_j| + |a_ij|) beyond the relative part.
                if prob.kind == "dense":
                    pat = absop((prob.A != 0).astype(float))
                elif prob.kind == "csr":
                    pat = absop(prob.m, prob.n, prob.indptr, prob.indices,
                                np.ones_like(prob.data))
                else:
                    pat = absop((prob.psf != 0).astype(float), prob.image_shape)
                ones = np.ones(nin)
                bound = bound + 2.0 ** -9 * (
                    (pat.rmatvec(np.abs(x)) + aop.rmatvec(ones)) if tr
                    else (pat.matvec(np.abs(x)) + aop.matvec(ones)))
            assert np.all(np.isfinite(y))
            assert np.all(np.abs(y - ref) <= bound), which
    finally:
        lib.lslu_op_destroy(op)


# ------------------------------------------------------------ solve parity

@pytest.mark.parametrize("kind", ["none", "wgcv", "gcv", "fixed", "optimal"])
def test_dense_blur_fp64(lib, ctx, kind):
    prob = config_problem("dense256")
    _compare(lib, ctx, prob, "fp64", 50, kind, relative=False, kappa_cap=1e5)


@pytest.mark.parametrize("shape,seed", [((40, 30), 1), ((30, 41), 2),
                                        ((67, 67), 3), ((130, 70), 4)])
@pytest.mark.parametrize("kind", ["none", "wgcv"])
def test_random_dense_fp64(lib, ctx, shape, seed, kind):
    prob = random_dense(*shape, seed=seed, nu=0.05)
    K = min(shape) - 5
    _compare(lib, ctx, prob, "fp64", K, kind, relative=True, kappa_cap=1e6)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tomography_small(lib, ctx, prec):
    prob = config_problem("tomo32")
    _compare(lib, ctx, prob, prec, 30, "wgcv", relative=True,
             check_free=(prec == "fp64"))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tomography_small_optimal(lib, ctx, prec):
    prob = config_problem("tomo32")
    _compare(lib, ctx, prob, prec, 30, "optimal", relative=True,
             check_free=(prec == "fp64"))


@pytest.mark.parametrize("prec,slack", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_optimal_error_not_above_wgcv(lib, ctx, prec, slack):
    """The basis does not depend on lambda, so at every k the optimal grid
    value (eq. lambda) gives an error to x_true no larger than the weighted
    GCV choice on the same grid."""
    prob = config_problem("tomo32")
    grid = lambda_grid()
    W = gpu_solve(lib, ctx, prob, prec, 30, "wgcv", grid=grid, grid_relative=True,
                  bases=False)
    O = gpu_solve(lib, ctx, prob, prec, 30, "optimal", grid=grid, grid_relative=True,
                  bases=False, x_true=prob.x_true)
    assert O["k_done"] == W["k_done"]
    assert np.array_equal(O["piv_t"], W["piv_t"]) and np.array_equal(O["piv_g"], W["piv_g"])
    nx = np.linalg.norm(prob.x_true)
    for k in range(1, O["k_done"] + 1):
        eo = np.linalg.norm(O["X"][:, k - 1] - prob.x_true) / nx
        ew = np.linalg.norm(W["X"][:, k - 1] - prob.x_true) / nx
        assert eo <= ew * (1 + slack) + slack, (k, eo, ew)
    assert 0 <= O["lambda_idx"][:O["k_done"]].min() and O["lambda_idx"][:O["k_done"]].max() < len(grid)


# ------------------------------------------------ sampled pivots (Sec. 2.2)

@pytest.mark.parametrize("name,prec,K,s", [("tomo32", "fp64", 30, 25), ("tomo32", "fp32", 30, 50),
                                           ("dense256", "fp64", 40, 25), ("deblur96", "fp64", 30, 100)])
def test_sampled_pivots(lib, ctx, name, prec, K, s):
    """The sampled-pivot variant against the oracle on the same candidate
    lists: pivots, x_k, H and W as for full pivoting (free and replay)."""
    from workloads import pivot_sample_lists
    prob = config_problem(name)
    rows = pivot_sample_lists(prob.m, prob.n, K, s, seed=11)
    relative = name != "dense256"
    R, G = _compare(lib, ctx, prob, prec, K, "wgcv", relative,
                    check_free=(prec == "fp64"), kappa_cap=1e5 if name == "dense256" else None,
                    pivot_sample=(rows, s))
    # the sample really decides: some pivots differ from full pivoting
    full = hybrid_lslu(make_operator(prob), prob.b, K, _reg("wgcv", relative))
    assert R.piv_t != full.piv_t[:len(R.piv_t)] or R.piv_g != full.piv_g[:len(R.piv_g)]


def test_sampled_pivots_listing_every_row_equal_full_pivoting(lib, ctx):
    """With every row listed and a sample as long as the list, the sampled
    search is the full search: bit-identical to the library's full run."""
    rng = np.random.default_rng(3)
    small = random_dense(60, 45, seed=9, nu=0.05)
    K = 20
    rows = np.full((2 * K + 1, 64), -1, dtype=np.int32)
    for i in range(2 * K + 1):
        length = small.m if i % 2 == 0 else small.n
        rows[i, :length] = rng.permutation(length)
    grid = lambda_grid()
    full = gpu_solve(lib, ctx, small, "fp64", K, "wgcv", grid=grid, grid_relative=True,
                     bases=False)
    samp = gpu_solve(lib, ctx, small, "fp64", K, "wgcv", grid=grid, grid_relative=True,
                     bases=False, pivot_sample=(rows, 64))
    assert np.array_equal(full["piv_t"], samp["piv_t"]) and np.array_equal(full["piv_g"], samp["piv_g"])
    assert np.array_equal(full["X"], samp["X"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_deblur_small(lib, ctx, prec):
    prob = config_problem("deblur96")
    _compare(lib, ctx, prob, prec, 40, "wgcv", relative=True,
             check_free=(prec == "fp64"))


@pytest.mark.parametrize("prec", ["bf16op", "fp16op"])
@pytest.mark.parametrize("name", ["deblur96", "tomo32"])
def test_16bit_operator_error(lib, ctx, prec, name):
    """The 16-bit operator modes (values and product inputs rounded to
    bfloat16 / binary16, sums and bases in float): exact pivot structure,
    and the error to x_true, stated against the FP64 oracle's."""
    prob = config_problem(name)
    op = make_operator(prob)
    K = 40 if name == "deblur96" else 30
    R = hybrid_lslu(op, prob.b, K, _reg("wgcv", True))
    G = gpu_solve(lib, ctx, prob, prec, K, "wgcv", grid=lambda_grid(),
                  grid_relative=True)
    check_basis_invariants(G, prob.m, prob.n)
    e_lo = np.array([rel(G["X"][:, k], prob.x_true) for k in range(G["k_done"])])
    e_64 = np.array([rel(R.X[:, k], prob.x_true) for k in range(R.k_done)])
    print(f"[{name} {prec}] rel err vs x_true: min {e_lo.min():.4f} at k={int(e_lo.argmin()) + 1}, "
          f"final {e_lo[-1]:.4f} (fp64 oracle: min {e_64.min():.4f}, final {e_64[-1]:.4f})")
    assert e_lo.min() < 1.5 * e_64.min()


def _fp8_cases():
    """Code points, midpoints (ties), values in the subnormal range, values
    past the largest finite one, both signs."""
    from gpu_helpers import e4m3
    pts = np.array([m * 2.0 ** -9 for m in range(8)]
                   + [(8 + mm) * 2.0 ** (e - 10) for e in range(1, 16) for mm in range(8)
                      if not (e == 15 and mm == 7)])
    mids = (pts[1:] + pts[:-1]) / 2
    rng = np.random.default_rng(11)
    extra = np.concatenate([rng.standard_normal(200) * 4, rng.uniform(0, 2.0 ** -6, 50),
                            [449.0, 463.9, 464.0, 1000.0, 3e5]])
    v = np.concatenate([pts, mids, extra])
    v = np.concatenate([v, -v]).astype(np.float32).astype(np.float64)
    assert np.all(np.abs(e4m3(v)) <= 448.0)
    return v


def _bf16(x):
    """bfloat16 rounding of float32 values (nearest, ties to even)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _16bit_cases():
    """Normal values of both signs, binary16 subnormals, and midpoints of
    both 16-bit formats near 1 (ties)."""
    rng = np.random.default_rng(12)
    v = np.concatenate([rng.standard_normal(300) * 4, rng.uniform(1e-7, 6e-5, 40),
                        1 + (2 * np.arange(20) + 1) / 2048.0, 1 + (2 * np.arange(20) + 1) / 256.0,
                        [0.0, 65504.0, 3.0e4]])
    v = np.concatenate([v, -v])
    return v.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16op", "fp16op", "fp8op"])
@pytest.mark.parametrize("kind", ["dense", "csr", "psf"])
def test_low_precision_rounding_is_exact(lib, ctx, kind, prec):
    """The 16- and 8-bit operator modes: the operator's values (rounded on the
    host; bfloat16 through float) and the product's input (rounded in the
    kernel) follow the format exactly.  A product of two such values is exact
    in float, so a diagonal operator diag(a) applied to x gives
    round(a) * round(x) to the bit."""
    import torch
    from gpu_helpers import e4m3
    rnd = {"bf16op": _bf16, "fp8op": e4m3,
           "fp16op": lambda z: np.asarray(z, np.float64).astype(np.float16).astype(np.float64)}[prec]
    v = _fp8_cases() if prec == "fp8op" else _16bit_cases()
    n = len(v)
    a = np.roll(v, 17)
    if kind == "dense":
        op = lib.lslu_op_dense(ctx, np.diag(a), lib.PRECISIONS[prec])
    elif kind == "csr":
        op = lib.lslu_op_csr(ctx, n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), a,
                             lib.PRECISIONS[prec])
    else:  # a 1x1 PSF is a scalar multiple of the identity
        a = np.full(n, 0.8125)
        op = lib.lslu_op_psf(ctx, 1, n, np.array([[0.8125]]), lib.PRECISIONS[prec])
    try:
        for tr in (0, 1):
            xt = torch.tensor(v, dtype=torch.float32, device="cuda")
            yt = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
            lib.lslu_op_apply(ctx, op, tr, xt, yt)
            torch.cuda.synchronize()
            y = yt.double().cpu().numpy()
            ref = rnd(a) * rnd(v)
            bad = np.flatnonzero(y != ref)
            assert bad.size == 0, (kind, tr, [(a[i], v[i], y[i], ref[i]) for i in bad[:5]])
    finally:
        lib.lslu_op_destroy(op)


@pytest.mark.parametrize("kind", ["dense", "csr", "psf"])
def test_fp32_operator_values_are_float(lib, ctx, kind):
    """FP32 operators hold float values and sum in double: diag(a) (a 1x1 PSF
    for the stencil) applied to float x gives float(float(a) * x) to the bit.
    The weight 0.3 is not a float, so an operator that kept the given double
    differs from this on about half of the entries."""
    import torch
    v = _16bit_cases()
    n = len(v)
    w = 0.3
    a = np.full(n, w)
    if kind == "dense":
        op = lib.lslu_op_dense(ctx, np.diag(a), lib.LSLU_FP32)
    elif kind == "csr":
        op = lib.lslu_op_csr(ctx, n, n, np.arange(n + 1), np.arange(n, dtype=np.int32), a,
                             lib.LSLU_FP32)
    else:
        op = lib.lslu_op_psf(ctx, 1, n, np.array([[w]]), lib.LSLU_FP32)
    try:
        ref = (np.float32(w).astype(np.float64) * v).astype(np.float32).astype(np.float64)
        unrounded = (w * v).astype(np.float32).astype(np.float64)
        assert np.count_nonzero(ref != unrounded) > n // 4  # the case tells the two apart
        for tr in (0, 1):
            xt = torch.tensor(v, dtype=torch.float32, device="cuda")
            yt = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
            lib.lslu_op_apply(ctx, op, tr, xt, yt)
            torch.cuda.synchronize()
            y = yt.double().cpu().numpy()
            bad = np.flatnonzero(y != ref)
            assert bad.size == 0, (kind, tr, [(v[i], y[i], ref[i]) for i in bad[:5]])
    finally:
        lib.lslu_op_destroy(op)


@pytest.mark.parametrize("name", ["deblur96", "tomo32"])
def test_8bit_operator_error(lib, ctx, name):
    """The E4M3 operator mode (values and product inputs with 3 fraction
    bits, sums and bases in float): exact pivot structure, and the error to
    x_true stated against the FP64 oracle's (looser than the 16-bit modes:
    each operator entry carries up to 6 % rounding)."""
    prob = config_problem(name)
    op = make_operator(prob)
    K = 40 if name == "deblur96" else 30
    R = hybrid_lslu(op, prob.b, K, _reg("wgcv", True))
    G = gpu_solve(lib, ctx, prob, "fp8op", K, "wgcv", grid=lambda_grid(), grid_relative=True)
    check_basis_invariants(G, prob.m, prob.n)
    e_lo = np.array([rel(G["X"][:, k], prob.x_true) for k in range(G["k_done"])])
    e_64 = np.array([rel(R.X[:, k], prob.x_true) for k in range(R.k_done)])
    print(f"[{name} fp8op] rel err vs x_true: min {e_lo.min():.4f} at k={int(e_lo.argmin()) + 1}, "
          f"final {e_lo[-1]:.4f} (fp64 oracle: min {e_64.min():.4f}, final {e_64[-1]:.4f})")
    assert e_lo.min() < 3.0 * e_64.min()


@pytest.mark.parametrize("prec", ["fp16op", "fp8op", "bf16op"])
def test_dense_matrix_core_modes(lib, ctx, prec):
    """The dense operator of the 256 x 256 problem (K = 50) in the 16- and
    8-bit modes, whose products run on the matrix cores (row lengths are
    multiples of the instruction's 16 or 32).  Each product takes the
    operator's rounded values and inputs rounded to the format, so the
    Hessenberg relations hold for the rounded operator and the rounded
    basis vectors to float rounding (every term exact in float):
    A_r round(L_k) = D_{k+1} H and A_r^T round(D_k) = L_k W within
    10 k 2^-24 of the magnitudes; the error to x_true is stated against the
    FP64 oracle's."""
    from gpu_helpers import e4m3
    prob = config_problem("dense256")
    K = 50
    rnd = {"fp16op": lambda z: np.asarray(z, np.float64).astype(np.float16).astype(np.float64),
           "fp8op": e4m3, "bf16op": _bf16}[prec]
    G = gpu_solve(lib, ctx, prob, prec, K, "wgcv", grid=lambda_grid(), grid_relative=True)
    check_basis_invariants(G, prob.m, prob.n)
    k = min(G["n_l"], G["n_d"] - 1)
    assert k >= 20
    Ar = rnd(prob.A)
    L, D = G["L"][:, :k], G["D"][:, :k + 1]
    H, W = G["H"][:k + 1, :k], G["W"][:k, :k]
    Lr, Dr = rnd(L), rnd(D[:, :k])
    u = 2.0 ** -24
    r1 = np.abs(Ar @ Lr - D @ H)
    b1 = 10 * k * u * (np.abs(Ar) @ np.abs(Lr) + np.abs(D) @ np.abs(H))
    r2 = np.abs(Ar.T @ Dr - L @ W)
    b2 = 10 * k * u * (np.abs(Ar.T) @ np.abs(Dr) + np.abs(L) @ np.abs(W))
    print(f"[dense256 {prec}] relations over k = {k}: max ratio to the bound "
          f"{(r1 / b1).max():.3f}, {(r2 / b2).max():.3f}")
    assert np.all(r1 <= b1) and np.all(r2 <= b2)
    R = hybrid_lslu(make_operator(prob), prob.b, K, _reg("wgcv", True))
    e_lo = np.array([rel(G["X"][:, j], prob.x_true) for j in range(G["k_done"])])
    e_64 = np.array([rel(R.X[:, j], prob.x_true) for j in range(R.k_done)])
    print(f"[dense256 {prec}] rel err vs x_true: min {e_lo.min():.4f} at k={int(e_lo.argmin()) + 1} "
          f"(FP64 oracle: min {e_64.min():.4f} at k={int(e_64.argmin()) + 1})")
    assert e_lo.min() < (3.0 if prec == "fp8op" else 1.5) * e_64.min()


# -------------------------------------------------------------- edge cases

def test_scaled_identity_breaks_down_at_one(lib, ctx):
    from workloads.problems import Problem
    n = 70
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    prob = Problem("cI", "dense", n, n, np.zeros(n), b, 0.0, A=2.5 * np.eye(n))
    for kind, lam in (("none", 0.0), ("fixed", 0.7)):
        G = gpu_solve(lib, ctx, prob, "fp64", 5, kind, lam)
        assert G["status"] == lib.LSLU_BREAKDOWN_U and G["k_done"] == 1
        assert np.allclose(G["x"], 2.5 * b / (2.5 ** 2 + lam ** 2), rtol=1e-14, atol=0)


def test_zero_rhs_and_adjoint_nullspace(lib, ctx):
    from workloads.problems import Problem
    A = np.zeros((5, 3))
    A[:3, :3] = np.eye(3)
    prob = Problem("z", "dense", 5, 3, np.zeros(3), np.zeros(5), 0.0, A=A)
    G = gpu_solve(lib, ctx, prob, "fp64", 2)
    assert G["status"] == lib.LSLU_ZERO_RHS and G["k_done"] == 0
    assert np.all(G["x"] == 0)
    prob.b = np.array([0.0, 0.0, 0.0, 1.0, -2.0])
    G = gpu_solve(lib, ctx, prob, "fp64", 2)
    assert G["status"] == lib.LSLU_BREAKDOWN_Q and G["k_done"] == 0
    assert np.all(G["x"] == 0)


@pytest.mark.parametrize("n,seed", [(5, 52), (8, 54), (70, 55)])
def test_square_consistent_system_solved_at_full_dimension(lib, ctx, n, seed):
    from workloads.problems import Problem
    rng = np.random.default_rng(seed)
    while True:
        A = rng.integers(-3, 4, size=(n, n)).astype(float) + (4 + n / 4) * np.eye(n)
        if np.linalg.cond(A) < 100:
            break
    x_true = rng.integers(-3, 4, size=n).astype(float)
    prob = Problem("sq", "dense", n, n, x_true, A @ x_true, 0.0, A=A)
    G = gpu_solve(lib, ctx, prob, "fp64", n)
    assert G["status"] == lib.LSLU_BREAKDOWN_U and G["k_done"] == n
    assert rel(G["x"], x_true) <= 1e-11


def test_maxiter_beyond_dimension_and_x0(lib, ctx):
    prob = random_dense(24, 9, seed=8, nu=0.05)
    rng = np.random.default_rng(9)
    x0 = rng.standard_normal(9)
    op = make_operator(prob)
    R = hybrid_lslu(op, prob.b, 10, RegParam("none"), x0=x0)
    G = gpu_solve(lib, ctx, prob, "fp64", 10, x0=x0)
    assert G["status"] == R.status == Status.BREAKDOWN_Q
    assert G["k_done"] == R.k_done == 9
    assert rel(G["x"], R.x) <= 1e-10


def test_early_stop_selects_k_stop(lib, ctx):
    prob = config_problem("dense256")
    op = make_operator(prob)
    R = hybrid_lslu(op, prob.b, 30, _reg("wgcv", False), stop_tol=1e-2,
                    early_stop=True)
    G = gpu_solve(lib, ctx, prob, "fp64", 30, "wgcv", grid=lambda_grid(),
                  early_stop=True, stop_tol=1e-2)
    assert G["k_stop"] == R.k_stop
    assert rel(G["x"], R.x) <= 1e-10


def test_ragged_sizes_and_determinism(lib, ctx):
    prob = tomography(13, 7, 19, 0.02, seed=12)
    a = gpu_solve(lib, ctx, prob, "fp64", 12, "wgcv", grid=lambda_grid(),
                  grid_relative=True)
    b = gpu_solve(lib, ctx, prob, "fp64", 12, "wgcv", grid=lambda_grid(),
                  grid_relative=True)
    assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["H"], b["H"])
    assert np.array_equal(a["L"], b["L"]) and np.array_equal(a["D"], b["D"])
    op = make_operator(prob)
    R = hybrid_lslu(op, prob.b, 12, _reg("wgcv", True))
    k_ok = well_separated_prefix(R, TAU["fp64"], 12)
    for k in range(1, k_ok + 1):
        assert rel(a["X"][:, k - 1], R.X[:, k - 1]) <= 1e-10


def test_invalid_options_are_rejected(lib, ctx):
    import torch
    prob = random_dense(10, 8, seed=1)
    op = lib.make_operator(ctx, prob, lib.LSLU_FP64)
    b = torch.tensor(prob.b, device="cuda")
    try:
        for kw in (dict(maxiter=0), dict(maxiter=20),
                   dict(maxiter=3, reg="wgcv"),
                   dict(maxiter=3, reg="optimal", grid=[0.1, 1.0]),
                   dict(maxiter=3, reg="wgcv", grid=[1.0, 0.5]),
                   dict(maxiter=3, reg="fixed", lam=-1.0),
                   dict(maxiter=2, pivot_sample=(np.zeros((5, 4), np.int32), 0)),
                   dict(maxiter=2, pivot_sample=(np.full((5, 4), 10, np.int32), 2))):
            K = kw.pop("maxiter")
            with pytest.raises(lib.LsluError) as ei:
                lib.lslu_solve(ctx, op, b, K, **kw)
            assert ei.value.status == lib.LSLU_EINVAL
        with pytest.raises(lib.LsluError):
            lib.lslu_op_dense(ctx, np.full((2, 2), np.nan))
        for bad in (-1, 5):  # precision modes are 0 (FP64) .. 4 (FP8 operator)
            for make in (lambda pr: lib.lslu_op_dense(ctx, np.eye(3), pr),
                         lambda pr: lib.lslu_op_csr(ctx, 2, 2, np.array([0, 1, 2]),
                                                    np.array([0, 1], np.int32),
                                                    np.ones(2), pr),
                         lambda pr: lib.lslu_op_psf(ctx, 4, 4, np.ones((3, 3)), pr)):
                with pytest.raises(lib.LsluError) as ei:
                    make(bad)
                assert ei.value.status == lib.LSLU_EINVAL
        # malformed CSR structure, each rejected before any entry past nnz
        # (or past a row's end) is read
        ix = np.array([0, 1, 2, 3, 4], np.int32)
        for ip, idx, why in (([0, 100, 5], ix, "exceeds nnz"),
                             ([0, 2, 1, 5], ix, "decreases"),
                             ([0, 2, 5], np.array([0, 9, 1, 2, 3], np.int32), "out of range"),
                             ([0, 2, 5], np.array([1, 0, 1, 2, 3], np.int32), "increasing")):
            with pytest.raises(lib.LsluError) as ei:
                lib.lslu_op_csr(ctx, len(ip) - 1, 6, np.array(ip), idx, np.ones(5))
            assert ei.value.status == lib.LSLU_EINVAL and why in str(ei.value), str(ei.value)
    finally:
        lib.lslu_op_destroy(op)


def test_graph_replays_match_eager(lib, ctx):
    """The captured graph of a solve, replayed several times with eager solves
    and other device work in between, gives bit-identical results each time."""
    import torch
    prob = config_problem("tomo32")
    op = lib.make_operator(ctx, prob, lib.LSLU_FP64)
    grid = lambda_grid()
    try:
        b = torch.tensor(prob.b, dtype=torch.float64, device="cuda")
        kw = dict(op=op, b=b, grid=grid, grid_relative=True, bases=False)
        ref = gpu_solve(lib, ctx, prob, "fp64", 20, "wgcv", eager=True, **kw)
        for rep in range(4):
            G = gpu_solve(lib, ctx, prob, "fp64", 20, "wgcv", **kw)
            assert np.array_equal(G["X"], ref["X"]) and np.array_equal(G["H"], ref["H"])
            assert np.array_equal(G["lambda_k"], ref["lambda_k"])
            assert list(G["piv_t"]) == list(ref["piv_t"])
            # other work in between: an eager solve of a different problem and
            # a torch kernel overwriting b, then b restored
            other = random_dense(30, 20, seed=rep)
            gpu_solve(lib, ctx, other, "fp64", 5, eager=True, bases=False)
            b.mul_(3.0)
            torch.cuda.synchronize()
            b.copy_(torch.tensor(prob.b, dtype=torch.float64, device="cuda"))
        # a changed right-hand side in the same buffer is picked up by replays
        b.mul_(2.0)
        G2 = gpu_solve(lib, ctx, prob, "fp64", 20, "wgcv", **kw)
        assert np.allclose(G2["X"], 2.0 * ref["X"], rtol=1e-12, atol=0)
    finally:
        lib.lslu_op_destroy(op)


def test_graph_cache_never_replays_a_destroyed_operator(lib, ctx):
    """Operators of the same shape created and destroyed in turn (their host
    handles and device arrays are often allocated where the previous ones
    lived), each solved with the same b, X and x_out buffers: every captured
    solve must use its own operator, i.e. match an eager solve of it."""
    import torch
    b = torch.zeros(40, dtype=torch.float64, device="cuda")
    X = torch.zeros((8, 30), dtype=torch.float64, device="cuda")
    x = torch.zeros(30, dtype=torch.float64, device="cuda")
    for seed in range(5):
        prob = random_dense(40, 30, seed=100 + seed, nu=0.01)
        b.copy_(torch.tensor(prob.b, dtype=torch.float64))
        # an operator of another size first, so that the device arrays of
        # this one move while its host handle may take the previous address
        spacer = lib.make_operator(ctx, random_dense(20 + 7 * seed, 10, seed=seed),
                                   lib.LSLU_FP64)
        op = lib.make_operator(ctx, prob, lib.LSLU_FP64)
        try:
            lib.lslu_solve(ctx, op, b, 8, reg="fixed", lam=0.05, X=X, x_out=x)
            torch.cuda.synchronize()
            got = X.clone()
            lib.lslu_solve(ctx, op, b, 8, reg="fixed", lam=0.05, X=X, x_out=x, eager=True)
            torch.cuda.synchronize()
            assert torch.equal(got, X), seed
        finally:
            lib.lslu_op_destroy(op)
            lib.lslu_op_destroy(spacer)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_host_array_solve_matches_device_solve(lib, ctx, prec):
    """lslu_solve_host: FP64 host arrays in and out, converted to the working
    precision exactly as a device tensor of that precision would be."""
    import torch
    prob = config_problem("tomo32")
    dt = torch.float64 if prec == "fp64" else torch.float32
    op = lib.make_operator(ctx, prob, lib.PRECISIONS[prec])
    try:
        x0 = np.random.default_rng(3).standard_normal(prob.n) * 0.01
        grid = lambda_grid()
        sh, xh, ih = lib.lslu_solve(ctx, op, prob.b, 15, reg="wgcv", grid=grid,
                                    grid_relative=True, x0=x0)
        b = torch.tensor(prob.b, dtype=dt, device="cuda")
        x0d = torch.tensor(x0, dtype=dt, device="cuda")
        sd, xd, idd = lib.lslu_solve(ctx, op, b, 15, reg="wgcv", grid=grid,
                                     grid_relative=True, x0=x0d)
        torch.cuda.synchronize()
        assert sh == sd and ih["k_done"] == idd["k_done"]
        assert np.array_equal(ih["piv_t"], idd["piv_t"]) and np.array_equal(ih["H"], idd["H"])
        assert np.array_equal(xh, xd.double().cpu().numpy())
        # repeated calls reuse the staging buffers (and the captured solve)
        sh2, xh2, _ = lib.lslu_solve(ctx, op, prob.b, 15, reg="wgcv", grid=grid,
                                     grid_relative=True, x0=x0)
        assert np.array_equal(xh, xh2)
        bad = prob.b.copy()
        bad[3] = np.nan
        with pytest.raises(lib.LsluError) as ei:
            lib.lslu_solve(ctx, op, bad, 15, reg="wgcv", grid=grid, grid_relative=True)
        assert ei.value.status == lib.LSLU_ENONFINITE
    finally:
        lib.lslu_op_destroy(op)


@pytest.mark.parametrize("reg", ["wgcv", "fixed", "none"])
def test_projected_problems_up_to_k200(lib, ctx, reg):
    """The projected problems at large k, where the (k+1) x k working matrix
    no longer fits in LDS and its first columns live in global scratch
    (k > 134; at k = 200 most of them): lambda_k, Ghat(k) and y_k of the
    library against the oracle's SVD solution of eq. TSP for the library's
    own H and beta (Section 3.2.1), at every k from 120 to 200."""
    from oracle.projected import ghat_value, projected_svd, select_lambda, tikhonov_coeffs
    prob = random_dense(230, 215, seed=41, nu=0.01)
    K = 200
    grid = lambda_grid()
    G = gpu_solve(lib, ctx, prob, "fp64", K, reg, lam=0.05, grid=grid, grid_relative=True,
                  bases=False)
    assert G["k_done"] == K
    rp = RegParam(reg, lam=0.05, grid=grid, grid_relative=True)
    worst_y = worst_g = 0.0
    for k in range(120, K + 1):
        s, c, V = projected_svd(G["H"][:k + 1, :k])
        lam, li, sep, _ = select_lambda(rp, k, prob.m, G["beta"], s, c, V, None, None)
        if sep > TAU["fp64"]:
            assert G["lambda_idx"][k - 1] == li, k
        y = tikhonov_coeffs(G["beta"], s, c, V, G["lambda_k"][k - 1])
        worst_y = max(worst_y, rel(G["Y"][:k, k - 1], y))
        gh = ghat_value(k, prob.n, prob.m, G["beta"], s, c, G["lambda_k"][k - 1])
        worst_g = max(worst_g, abs(G["ghat"][k - 1] - gh) / abs(gh))
        if reg == "wgcv":
            assert np.isclose(G["lambda_k"][k - 1], s[0] * grid[G["lambda_idx"][k - 1]],
                              rtol=1e-12)
    kap = s[0] / s[-1]
    print(f"[projected k<=200 {reg}] max y error {worst_y:.2e}, max Ghat error {worst_g:.2e}, "
          f"kappa(H) at k=200 {kap:.1e}")
    # y_k of a Tikhonov problem is as accurate as its conditioning allows:
    # kappa(H) u for lambda = 0, less with damping
    assert worst_y <= 1e-13 * max(kap, 1.0) and worst_y <= 1e-6
    assert worst_g <= 1e-8


# ------------------------------------- coefficients published in chunks

@pytest.mark.parametrize("cols", [46, 45])
def test_psf_coefficient_chunks(lib, ctx, cols):
    """140 iterations, so a launch eliminates up to 140 earlier basis
    vectors: the lead publishes their coefficients in three 64-slot chunks
    as its triangular solve finishes each, and a PSF consumer's elimination
    waits chunk by chunk.  Even width (pixel pairs per lane) and odd width
    (one pixel per lane): FP64 free (every pivot) and replayed and FP32
    replayed against the oracle (x_k, H, W at every k); BF16-op (matrix-core
    products) through the Hessenberg relations of its own bases (eq. nhr,
    eq. nhr2), to the rounding of its bfloat16 products, which a coefficient
    staged late or from the wrong slot would break by far."""
    from oracle.operators import PsfOp
    prob = psf_deblur(36, 2, 1.0, 0.01, seed=21, cols=cols)
    K = 140
    for prec in ("fp64", "fp32"):
        # every pivot search is well separated here, so the free run is held
        # to the oracle's pivots at every k
        R, G = _compare(lib, ctx, prob, prec, K, "wgcv", True, check_free=(prec == "fp64"))
        assert G["k_done"] == K
    G = gpu_solve(lib, ctx, prob, "bf16op", K, "wgcv", grid=lambda_grid(), grid_relative=True)
    check_basis_invariants(G, prob.m, prob.n)
    op = make_operator(prob)
    aop = PsfOp(np.abs(prob.psf), prob.image_shape)
    k = min(G["n_l"], G["n_d"] - 1)
    assert k >= 129
    L, D = G["L"][:, :k], G["D"][:, :k + 1]
    H, W = G["H"][:k + 1, :k], G["W"][:k, :k]
    ub, uf = 2.0 ** -8, 2.0 ** -24
    worst = 0.0
    for j in range(k):
        # column j of A L_k = D_{k+1} H and of A^T D_k = L_k W: the product
        # rounds operator and input to bfloat16 (2 ub |A||x|), the sums and
        # stored vectors are float
        r1 = np.linalg.norm(op.matvec(L[:, j]) - D @ H[:, j])
        b1 = 2.5 * ub * np.linalg.norm(aop.matvec(np.abs(L[:, j]))) \
            + 10 * k * uf * np.linalg.norm(np.abs(D) @ np.abs(H[:, j]))
        r2 = np.linalg.norm(op.rmatvec(D[:, j]) - L @ W[:, j])
        b2 = 2.5 * ub * np.linalg.norm(aop.rmatvec(np.abs(D[:, j]))) \
            + 10 * k * uf * np.linalg.norm(np.abs(L) @ np.abs(W[:, j]))
        assert r1 <= b1 and r2 <= b2, (j, r1 / b1, r2 / b2)
        worst = max(worst, r1 / b1, r2 / b2)
    print(f"[chunks {prob.name}] bf16op relations at most {worst:.2f} of their rounding bound")
