"""Pins of the oracle's derivatives of x_k (oracle/gradient.py).

The complex-step derivative is pinned to things other than itself:
* at real input the fixed-pivot recurrence reproduces ``hybrid_lslu`` (the
  pinned forward oracle) with the same pivots;
* central finite differences of ``hybrid_lslu`` itself, in directions where
  the oracle's own pivot searches do not change;
* the closed form at full dimension: for a square nonsingular A, LSLU with
  lambda = 0 gives x_n = A^{-1} b (Algorithm 5 terminates), so
  (d x_n / d b)^T xbar = A^{-T} xbar;
* the lambda derivative of the squared error against ``dloss_dlambda``
  (pinned against central differences through the SVD form of eq. TSP).
"""

import numpy as np
import pytest

from oracle import RegParam, make_operator
from oracle.gradient import (fixed_pivot_lslu, vjp_directional, vjp_full,
                             vjp_lambda)
from oracle.hessenberg import Status, hybrid_lslu
from oracle.projected import dloss_dlambda, projected_svd
from workloads import psf_deblur, random_dense, tomography


def _problems():
    return [
        random_dense(40, 30, seed=3, nu=0.01),
        random_dense(25, 35, seed=4, nu=0.01),
        tomography(16, 12, 23, 0.02, seed=5),
        psf_deblur(12, 3, 1.5, 0.01, seed=6),
    ]


@pytest.mark.parametrize("idx", range(4))
def test_fixed_pivot_recurrence_reproduces_hybrid_lslu(idx):
    prob = _problems()[idx]
    op = make_operator(prob)
    K, lam = 10, 0.05
    R = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam))
    for k in (1, 4, K):
        x = fixed_pivot_lslu(op, prob.b, k, lam, R.piv_t, R.piv_g)
        ref = R.X[:, k - 1]
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max(), k


@pytest.mark.parametrize("idx", range(4))
def test_complex_step_against_central_differences(idx):
    prob = _problems()[idx]
    op = make_operator(prob)
    K, lam = 10, 0.05
    reg = RegParam("fixed", lam=lam)
    R = hybrid_lslu(op, prob.b, K, reg)
    rng = np.random.default_rng(idx)
    xbar = rng.standard_normal(prob.n)
    h = 1e-6 * np.linalg.norm(prob.b)
    checked = 0
    for _ in range(3):
        v = rng.standard_normal(prob.m)
        v /= np.linalg.norm(v)
        Rp = hybrid_lslu(op, prob.b + h * v, K, reg)
        Rm = hybrid_lslu(op, prob.b - h * v, K, reg)
        if Rp.piv_t != R.piv_t or Rm.piv_t != R.piv_t or Rp.piv_g != R.piv_g \
                or Rm.piv_g != R.piv_g:
            continue  # a pivot moved: the map is not smooth along v here
        fd = xbar @ (Rp.X[:, K - 1] - Rm.X[:, K - 1]) / (2 * h)
        cs = vjp_directional(op, prob.b, K, lam, R.piv_t, R.piv_g, xbar, v)
        scale = np.linalg.norm(xbar) * np.linalg.norm(
            (Rp.X[:, K - 1] - Rm.X[:, K - 1]) / (2 * h)) + abs(fd)
        assert abs(cs - fd) <= 1e-6 * scale, (cs, fd)
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("seed", [5, 7])
def test_full_dimension_gradient_is_inverse_transpose(seed):
    prob = random_dense(12, 12, seed=seed)
    op = make_operator(prob)
    R = hybrid_lslu(op, prob.b, 12)
    assert R.k_done == 12 and R.status == Status.BREAKDOWN_U  # d-side ends at k = m
    A = prob.A
    x = fixed_pivot_lslu(op, prob.b, 12, 0.0, R.piv_t, R.piv_g)
    assert np.allclose(x, np.linalg.solve(A, prob.b), rtol=0, atol=1e-9 * np.abs(x).max())
    xbar = np.random.default_rng(seed).standard_normal(12)
    g = vjp_full(op, prob.b, 12, 0.0, R.piv_t, R.piv_g, xbar)
    ex = np.linalg.solve(A.T, xbar)
    kappa = np.linalg.cond(A)
    assert np.abs(g - ex).max() <= 1e2 * kappa * kappa * np.finfo(float).eps * np.abs(ex).max()


@pytest.mark.parametrize("lam", [0.01, 0.2])
def test_lambda_derivative_matches_dloss_dlambda(lam):
    prob = random_dense(40, 30, seed=3, nu=0.01)
    op = make_operator(prob)
    K = 12
    R = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam))
    for k in (3, 8, 12):
        xk = fixed_pivot_lslu(op, prob.b, k, lam, R.piv_t, R.piv_g)
        xbar = 2.0 * (xk - prob.x_true)
        cs = vjp_lambda(op, prob.b, k, lam, R.piv_t, R.piv_g, xbar)
        s, c, V = projected_svd(R.H[:k + 1, :k])
        ref = dloss_dlambda(R.beta, s, c, V, lam, R.L[:, :k], np.zeros(prob.n), prob.x_true)
        assert abs(cs - ref) <= 1e-9 * max(abs(ref), 1e-12), (k, cs, ref)


def test_lambda_derivative_against_central_differences():
    prob = psf_deblur(12, 3, 1.5, 0.01, seed=6)
    op = make_operator(prob)
    K, lam, h = 10, 0.05, 1e-6
    R = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam))
    xbar = np.random.default_rng(1).standard_normal(prob.n)
    cs = vjp_lambda(op, prob.b, K, lam, R.piv_t, R.piv_g, xbar)
    xp = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam + h)).X[:, K - 1]
    xm = hybrid_lslu(op, prob.b, K, RegParam("fixed", lam=lam - h)).X[:, K - 1]
    fd = xbar @ (xp - xm) / (2 * h)
    assert abs(cs - fd) <= 1e-6 * (np.linalg.norm(xbar) * np.linalg.norm((xp - xm) / (2 * h))), (cs, fd)
