"""lslu_solve_static, the solve for callers that cannot allocate device
memory, against lslu_solve: several calls in a row on one context, each
smaller than the one before, each compared with lslu_solve of the same
problem (same kernels, so every output must be bit-identical); a solve too
large for the fixed workspace is refused; the reverse pass and basis copies
do not apply after such a solve."""

import numpy as np
import pytest

from workloads import lambda_grid, psf_deblur, random_dense, tomography

pytestmark = pytest.mark.gpu

KEYS = ("piv_t", "piv_g", "own_piv_t", "own_piv_g", "H", "W", "Y", "lambda_k",
        "lambda_idx", "ghat", "sep_lambda", "sigma_max", "sigma_min")


def _pair(lib, ctx, prob, prec, K, with_X=True, **kw):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    op = lib.make_operator(ctx, prob, lib.PRECISIONS[prec])
    try:
        b = torch.tensor(prob.b, dtype=dt, device="cuda")
        Xa = torch.zeros((K, prob.n), dtype=dt, device="cuda") if with_X else None
        Xb = torch.full((K, prob.n), float("nan"), dtype=dt, device="cuda") if with_X else None
        print(f"[no-alloc] {prob.name} {prec} K={K} X={with_X} {sorted(kw)}", flush=True)
        sa, xa, ia = lib.lslu_solve(ctx, op, b, K, X=Xa, **kw)
        sb, xb, ib = lib.lslu_solve(ctx, op, b, K, X=Xb, static=True, **kw)
        torch.cuda.synchronize()
        assert sa == sb
        for key in ("k_done", "k_stop", "n_l", "n_d", "beta", "piv_t_mismatch",
                    "piv_g_mismatch"):
            assert ia[key] == ib[key], key
        for key in KEYS:
            assert np.array_equal(ia[key], ib[key], equal_nan=True), key
        assert torch.equal(xa, xb)
        if with_X:
            assert torch.equal(Xa, Xb)
        return ib
    finally:
        lib.lslu_op_destroy(op)


def test_static_solve_matches_solve(lib):
    from oracle import RegParam, make_operator
    from oracle.hessenberg import hybrid_lslu
    from gpu_helpers import replay_from
    ctx = lib.lslu_create(0)
    try:
        grid = lambda_grid()
        # decreasing sizes: each call leaves its contents in the shared array
        tomo = tomography(48, 48, 49, 0.02, seed=31)           # CSR, 2352 x 2304
        i1 = _pair(lib, ctx, tomo, "fp32", 40, reg="wgcv", grid=grid, grid_relative=True)
        blur = psf_deblur(40, 3, 1.5, 0.01, seed=33)            # PSF, 1600 x 1600
        _pair(lib, ctx, blur, "fp64", 25, reg="gcv", grid=grid, grid_relative=True)
        dense = random_dense(40, 30, seed=32, nu=0.02)          # dense, 40 x 30
        _pair(lib, ctx, dense, "fp64", 12, with_X=False, reg="fixed", lam=0.05)
        # replayed pivots and lambda indices (from the oracle), smaller still
        small = tomography(16, 12, 23, 0.02, seed=34)
        R = hybrid_lslu(make_operator(small), small.b, 10,
                        RegParam("wgcv", grid=grid, grid_relative=True))
        _pair(lib, ctx, small, "fp64", 10, reg="wgcv", grid=grid, grid_relative=True,
              **replay_from(R, 10))
        assert i1["k_done"] == 40
    finally:
        lib.lslu_destroy(ctx)


def test_static_solve_limits(lib):
    import torch
    from workloads import config_problem
    ctx = lib.lslu_create(0)
    prob = config_problem("tomo32")
    op = lib.make_operator(ctx, prob, lib.LSLU_FP64)
    try:
        b = torch.tensor(prob.b, dtype=torch.float64, device="cuda")
        lib.lslu_solve(ctx, op, b, 10, static=True)
        # the reverse pass and basis copies read the context's own workspace
        dst = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        assert lib.lib.lslu_get_basis(ctx, 0, 1, lib.c_void_p(dst.data_ptr())) == lib.LSLU_EINVAL
        assert lib.lib.lslu_vjp(ctx, op, 1, lib.c_void_p(dst.data_ptr()),
                                lib.c_void_p(b.data_ptr()), None) == lib.LSLU_EINVAL
        with pytest.raises(ValueError):
            lib.lslu_solve(ctx, op, b, 10, static=True, asynchronous=True)
    finally:
        lib.lslu_op_destroy(op)
    # 1024 x 1024 in FP32, 20 iterations: the bases alone take 168 MB
    big = psf_deblur(1024, 3, 1.5, 0.01, seed=35)
    op = lib.make_operator(ctx, big, lib.LSLU_FP32)
    try:
        b = torch.tensor(big.b, dtype=torch.float32, device="cuda")
        with pytest.raises(lib.LsluError) as ei:
            lib.lslu_solve(ctx, op, b, 20, static=True)
        assert ei.value.status == lib.LSLU_EINVAL and "MiB" in str(ei.value)
    finally:
        lib.lslu_op_destroy(op)
        lib.lslu_destroy(ctx)
