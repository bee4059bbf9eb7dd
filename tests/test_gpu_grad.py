"""The derivative in lambda of the squared error of x_k (LSLU_FLAG_GRAD_LAMBDA)
against the oracle's ``dloss_dlambda`` (Section 3.2.1, eq. TSP and eq. lambda)
and against central differences of the library's own iterates.

Scale of the comparison: by Cauchy-Schwarz |d loss/d lambda| is at most
2 ||x_k - x_true|| ||L_k dy/dlambda||; rounding in the contraction and in the
solves is relative to that bound, not to the derivative itself (which crosses
zero at the optimal lambda).
"""

import numpy as np
import pytest

from gpu_helpers import gpu_solve, replay_from
from oracle import RegParam, make_operator
from oracle.hessenberg import hybrid_lslu
from oracle.projected import (dloss_dlambda, projected_svd,
                              tikhonov_coeffs_dlambda)
from workloads import config_problem, lambda_grid, random_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.lslu_create(0)
    yield c
    lib.lslu_destroy(c)


def _oracle_grad(R, prob, k):
    Hk = R.H[:k + 1, :k]
    s, c, V = projected_svd(Hk)
    lam = float(R.lambdas[k - 1])
    Lk = R.L[:, :k]
    x0 = np.zeros(prob.n)
    g = dloss_dlambda(R.beta, s, c, V, lam, Lk, x0, prob.x_true)
    dy = tikhonov_coeffs_dlambda(R.beta, s, c, V, lam)
    bound = 2.0 * np.linalg.norm(R.X[:, k - 1] - prob.x_true) * np.linalg.norm(Lk @ dy)
    return g, bound


@pytest.mark.parametrize("name,kind,K", [
    ("dense64", "fixed", 20), ("dense64", "wgcv", 20),
    ("tomo32", "wgcv", 30), ("tomo32", "gcv", 30), ("tomo32", "optimal", 30),
    ("rand", "fixed", 25)])
def test_grad_lambda_matches_oracle_fp64(lib, ctx, name, kind, K):
    prob = (random_dense(90, 70, seed=4) if name == "rand"
            else config_problem("dense256") if name == "dense64"
            else config_problem("tomo32"))
    op = make_operator(prob)
    reg = RegParam(kind, lam=0.05, grid=lambda_grid(), grid_relative=True,
                   x_true=prob.x_true if kind == "optimal" else None)
    R = hybrid_lslu(op, prob.b, K, reg)
    Kr = min(K, R.k_done)
    grid = lambda_grid() if kind in ("wgcv", "gcv", "optimal") else None
    G = gpu_solve(lib, ctx, prob, "fp64", Kr, kind, 0.05, grid, True,
                  replay=replay_from(R, Kr), x_true=prob.x_true, grad_lambda=True,
                  bases=False)
    assert G["k_done"] == Kr
    worst = 0.0
    for k in range(1, Kr + 1):
        kap = G["sigma_max"][k - 1] / G["sigma_min"][k - 1]
        if kap > 1e8:
            break
        g, bound = _oracle_grad(R, prob, k)
        e = abs(G["dloss_dlambda"][k - 1] - g) / max(bound, 1e-300)
        worst = max(worst, e)
        assert e <= 1e-8, (k, G["dloss_dlambda"][k - 1], g, bound)
    print(f"[grad {prob.name} {kind}] worst error / bound {worst:.3e}")


def test_grad_lambda_is_zero_without_regularisation(lib, ctx):
    prob = config_problem("tomo32")
    G = gpu_solve(lib, ctx, prob, "fp64", 12, "none", x_true=prob.x_true,
                  grad_lambda=True, bases=False)
    assert np.all(G["lambda_k"][:G["k_done"]] == 0.0)
    assert np.all(G["dloss_dlambda"][:G["k_done"]] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grad_lambda_against_central_differences(lib, ctx, prec):
    """Fixed-lambda solves at lambda +- h: the basis does not depend on
    lambda, so the central difference of ||x_k - x_true||^2 over the
    library's own iterates approximates its derivative."""
    prob = config_problem("tomo32")
    K, lam = 25, 0.08
    h = lam * 1e-3
    runs = {}
    for l in (lam - h, lam, lam + h):
        runs[l] = gpu_solve(lib, ctx, prob, prec, K, "fixed", l, x_true=prob.x_true,
                            grad_lambda=True, bases=False)
    for k in range(2, runs[lam]["k_done"] + 1):
        lp = np.sum((runs[lam + h]["X"][:, k - 1] - prob.x_true) ** 2)
        lm = np.sum((runs[lam - h]["X"][:, k - 1] - prob.x_true) ** 2)
        fd = (lp - lm) / (2 * h)
        g = runs[lam]["dloss_dlambda"][k - 1]
        scale = max(abs(fd), abs(g), 1e-3 * np.sum(prob.x_true ** 2))
        tol = 1e-5 if prec == "fp64" else 2e-2
        assert abs(g - fd) <= tol * scale, (k, g, fd)


def test_grad_lambda_needs_x_true(lib, ctx):
    prob = random_dense(40, 30, seed=1)
    with pytest.raises(lib.LsluError) as ei:
        gpu_solve(lib, ctx, prob, "fp64", 5, "fixed", 0.1, grad_lambda=True,
                  bases=False)
    assert ei.value.status == lib.LSLU_EINVAL
