"""Forward sensitivity of the oracle's iterates, for per-step tolerances.

Rounding inside the recurrence acts like a small perturbation of the data at
every step, and the LU-type bases amplify it wherever a new basis vector is
the small difference of large ones; in the noise-dominated tail (lambda at the
grid minimum) the projected problem amplifies it further.  Two runs that
differ only in rounding order therefore agree on x_k to about
k * u * s_k, where s_k is the condition number of x_k with respect to relative
perturbations of A and b.  s_k is measured here with the oracle alone: perturb
A's stored values and b by a relative eps (uniform, seeded), rerun, and
re-solve the projected problem at the unperturbed lambda_k so that a flip
between two near-equal grid values does not count as sensitivity.

Only oracle functions are called; nothing here runs on the GPU.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from oracle import make_operator
from oracle.hessenberg import hybrid_lslu
from oracle.projected import projected_svd, tikhonov_coeffs


def _perturbed(prob, eps, seed):
    rng = np.random.default_rng(seed)

    def jig(v):
        return v * (1.0 + eps * rng.uniform(-1.0, 1.0, v.shape))

    kw = {"b": jig(prob.b)}
    if prob.kind == "dense":
        kw["A"] = jig(prob.A)
    elif prob.kind == "csr":
        kw["data"] = jig(prob.data)
    else:
        kw["psf"] = jig(prob.psf)
    return dataclasses.replace(prob, **kw)


def perturbed_runs(prob, R, reg, K, eps=1e-9, seeds=(1, 2)):
    """Oracle runs on copies of the problem with A's stored values and b
    perturbed by a relative eps; their pivots are required to equal R's (eps
    is far below every pivot separation the tests rely on, so the response is
    linear)."""
    runs = []
    for seed in seeds:
        P = _perturbed(prob, eps, seed)
        Rp = hybrid_lslu(make_operator(P), P.b, K, reg)
        if Rp.piv_g[:K] != R.piv_g[:K] or Rp.piv_t[:K + 1] != R.piv_t[:K + 1]:
            raise AssertionError("perturbation changed the pivots; lower eps")
        runs.append(Rp)
    return runs


def sensitivity_at(runs, lambdas, X_ref, K, eps=1e-9):
    """s_k, k = 1..K: the largest over the perturbed runs of
    ||x_k(perturbed) - x_k|| / (||x_k|| eps), each perturbed x_k re-solved at
    the given lambda_k (the bases do not depend on lambda, so any lambda
    sequence can be priced from the same runs)."""
    s = np.zeros(K)
    for Rp in runs:
        for k in range(1, min(K, Rp.k_done, X_ref.shape[1]) + 1):
            sv, c, V = projected_svd(Rp.H[:k + 1, :k])
            y = tikhonov_coeffs(Rp.beta, sv, c, V, lambdas[k - 1])
            xk = Rp.L[:, :k] @ y
            ref = X_ref[:, k - 1]
            s[k - 1] = max(s[k - 1], np.linalg.norm(xk - ref) / (np.linalg.norm(ref) * eps))
    return s


def forward_sensitivity(prob, R, reg, K, eps=1e-9, seeds=(1, 2)):
    """s_k of the iterates R.X at R's own lambda_k (see sensitivity_at)."""
    runs = perturbed_runs(prob, R, reg, K, eps, seeds)
    return sensitivity_at(runs, R.lambdas, R.X, min(K, R.k_done), eps)


def step_tolerances(s, u, stated):
    """Per-step bound: the stated tolerance, or 10 k u s_k where the problem's
    forward sensitivity does not allow the stated one."""
    k = np.arange(1, len(s) + 1)
    return np.maximum(stated, 10.0 * k * u * s)


def measured_prefix(prob, R, reg, K, u, stated, eps=1e-9, seeds=(1, 2)):
    """Largest k <= K at which the stated tolerance still applies by the
    oracle's measured forward sensitivity: 10 k' u s_k' <= stated for every
    k' <= k, with s_k the larger of the sensitivity of x_k (sensitivity_at)
    and of column k of H (max_j |H_p(j,k) - H(j,k)| / (max|H| eps)) over
    perturbed oracle runs.  A perturbed run whose pivots differ from R's
    ends the prefix where they first differ."""
    runs, stop = [], K
    for seed in seeds:
        P = _perturbed(prob, eps, seed)
        Rp = hybrid_lslu(make_operator(P), P.b, K, reg)
        for k in range(1, K + 1):
            if Rp.piv_g[:k] != R.piv_g[:k] or Rp.piv_t[:k + 1] != R.piv_t[:k + 1]:
                stop = min(stop, k - 1)
                break
        runs.append(Rp)
    kk = min(stop, R.k_done)
    if kk < 1:
        return 0
    sx = sensitivity_at(runs, R.lambdas, R.X, kk, eps)
    Hs = np.abs(R.H).max()
    sh = np.zeros(kk)
    for Rp in runs:
        d = np.abs(Rp.H[:kk + 1, :kk] - R.H[:kk + 1, :kk]).max(axis=0)
        sh = np.maximum(sh, d / (Hs * eps))
    k = np.arange(1, kk + 1)
    ok = 10.0 * k * u * np.maximum(sx, sh) <= stated
    return kk if ok.all() else int(np.argmin(ok))
