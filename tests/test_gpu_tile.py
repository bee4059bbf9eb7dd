"""Tile shapes of the PSF products (lslu_op_tile): every shape sums each
output pixel in the same order, so products and whole solves must be
bit-identical whichever shape is used or measured fastest."""

import numpy as np
import pytest

from workloads import psf_deblur, random_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.lslu_create(0)
    yield c
    lib.lslu_destroy(c)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16op", "fp8op"])
@pytest.mark.parametrize("shape", [(96, 96, 7), (40, 70, 3), (130, 33, 15)])
def test_tile_shapes_give_identical_results(lib, ctx, prec, shape):
    import torch
    rows, cols, hw = shape
    prob = psf_deblur(rows, hw, 1.5 + 0.1 * hw, 0.01, seed=31, cols=cols)
    dt = torch.float64 if prec == "fp64" else torch.float32
    op = lib.make_operator(ctx, prob, lib.PRECISIONS[prec])
    try:
        chosen = lib.lslu_op_tile(ctx, op, 0)
        assert chosen in (2, 4, 8)
        x = torch.tensor(np.random.default_rng(1).standard_normal(prob.n), dtype=dt, device="cuda")
        b = torch.tensor(prob.b, dtype=dt, device="cuda")
        outs = []
        for r in (2, 4, 8):
            assert lib.lslu_op_tile(ctx, op, r) == r
            ya = torch.zeros(prob.m, dtype=dt, device="cuda")
            yt = torch.zeros(prob.n, dtype=dt, device="cuda")
            lib.lslu_op_apply(ctx, op, 0, x, ya)
            lib.lslu_op_apply(ctx, op, 1, x, yt)
            X = torch.zeros((12, prob.n), dtype=dt, device="cuda")
            st, xo, info = lib.lslu_solve(ctx, op, b, 12, reg="fixed", lam=0.05, X=X)
            torch.cuda.synchronize()
            outs.append((ya.clone(), yt.clone(), X.clone(), list(info["piv_t"])))
        for o in outs[1:]:
            assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
            assert torch.equal(o[2], outs[0][2]) and o[3] == outs[0][3]
    finally:
        lib.lslu_op_destroy(op)


def test_tile_arguments(lib, ctx):
    prob = psf_deblur(32, 3, 1.5, 0.01, seed=2)
    op = lib.make_operator(ctx, prob, lib.PRECISIONS["fp32"])
    dense = lib.make_operator(ctx, random_dense(20, 10, seed=1), lib.PRECISIONS["fp64"])
    try:
        with pytest.raises(lib.LsluError) as ei:
            lib.lslu_op_tile(ctx, op, 3)
        assert ei.value.status == lib.LSLU_EINVAL
        with pytest.raises(lib.LsluError) as ei:
            lib.lslu_op_tile(ctx, dense, 0)
        assert ei.value.status == lib.LSLU_EUNSUPPORTED
    finally:
        lib.lslu_op_destroy(op)
        lib.lslu_op_destroy(dense)
