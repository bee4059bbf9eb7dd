"""Derivatives of the Hybrid LSLU iterate x_k with respect to b and lambda
(test infrastructure, like the rest of ``oracle``; nothing in the library
imports it).

With the pivots held fixed, the recurrence of Algorithm 5 is a composition of
operator products, eliminations with coefficients read at the pivot rows and
divisions by pivot entries: a smooth map of b (Alg. 5, Section 2).  The
projected problem of iteration k is the Tikhonov problem of eq. TSP,
    y_k = argmin ||beta e_1 - H_k y||^2 + lambda^2 ||y||^2
        = (H_k^T H_k + lambda^2 I)^{-1} H_k^T beta e_1,
and x_k = x_0 + L_k y_k (Section 3.2.1).  Near a point where every pivot
search is decided with room to spare, the pivots do not move under small
perturbations of b, so the derivative of x_k is the derivative of this
fixed-pivot map.

The reference derivative is the complex step (Squire and Trapp 1998; Martins,
Sturdza and Alonso 2003): for a real-analytic f,
    f'(b) v = Im f(b + i h v) / h + O(h^2),
with no cancellation, so h = 1e-30 gives it to rounding.  That needs the
forward map evaluated in complex arithmetic as an analytic function:
``fixed_pivot_lslu`` runs the recurrence with the given pivots (so no |.|
comparisons are taken on complex numbers) and solves the projected problem
through the normal equations with plain transposes (no conjugation), which is
analytic in the data.  At real input it computes the same x_k as
``hessenberg.hybrid_lslu`` with those pivots.
"""

from __future__ import annotations

import numpy as np


def _apply(f, v):
    """A real linear operator applied to a real or complex vector."""
    if np.iscomplexobj(v):
        return f(np.ascontiguousarray(v.real)) + 1j * f(np.ascontiguousarray(v.imag))
    return f(v)


def fixed_pivot_lslu(op, b, k, lam, piv_t, piv_g, x0=None):
    """x_k of Hybrid LSLU (Algorithm 5) with the row pivots ``piv_t``
    (t(1), t(2), ...) and column pivots ``piv_g`` (g(1), g(2), ...) given,
    lambda fixed.  ``b`` (and ``lam``) may be complex.  ``piv_t`` needs k+1
    entries unless the d-side breaks down at iteration k (k = m), in which case
    H(k+1, k) = 0 as in the oracle's recurrence."""
    m, n = op.shape
    dt = np.result_type(np.asarray(b).dtype, np.asarray(lam).dtype, np.float64)
    b = np.asarray(b, dtype=dt)
    x0v = np.zeros(n, dtype=dt) if x0 is None else np.asarray(x0, dtype=dt)
    r0 = b - _apply(op.matvec, x0v) if x0 is not None else b.copy()
    # r_0 and its pivot entry beta; d_1 = r_0 / beta
    beta = r0[piv_t[0]]
    D = [r0 / beta]
    L = []
    H = np.zeros((k + 1, k), dtype=dt)
    for kk in range(1, k + 1):
        # adjoint product, elimination of l_1..l_{kk-1} (coefficients W(j, kk)
        # read at the pivot rows g(j)), normalisation by the entry at g(kk)
        q = _apply(op.rmatvec, D[kk - 1])
        for j in range(1, kk):
            q = q - q[piv_g[j - 1]] * L[j - 1]
        L.append(q / q[piv_g[kk - 1]])
        # forward product, elimination of d_1..d_kk (coefficients H(j, kk)),
        # normalisation by H(kk+1, kk) = u(t(kk+1))
        u = _apply(op.matvec, L[kk - 1])
        for j in range(1, kk + 1):
            H[j - 1, kk - 1] = u[piv_t[j - 1]]
            u = u - H[j - 1, kk - 1] * D[j - 1]
        if kk < len(piv_t) and kk < m:
            H[kk, kk - 1] = u[piv_t[kk]]
            D.append(u / H[kk, kk - 1])
        elif kk < k:
            raise ValueError("the d-side breaks down before iteration k")
    # projected Tikhonov problem (eq. TSP) by the normal equations, plain
    # transposes so that the map stays analytic
    c = np.zeros(k + 1, dtype=dt)
    c[0] = beta
    M = H.T @ H + (lam * lam) * np.eye(k)
    y = np.linalg.solve(M, H.T @ c)
    return x0v + np.stack(L, axis=1) @ y


def vjp_directional(op, b, k, lam, piv_t, piv_g, xbar, v, x0=None, h=1e-30):
    """xbar^T (d x_k / d b) v by one complex step."""
    xk = fixed_pivot_lslu(op, np.asarray(b, np.float64) + 1j * h * np.asarray(v, np.float64),
                          k, lam, piv_t, piv_g, x0)
    return float(np.dot(np.asarray(xbar, np.float64), xk.imag) / h)


def vjp_lambda(op, b, k, lam, piv_t, piv_g, xbar, x0=None, h=1e-30):
    """xbar^T (d x_k / d lambda) by one complex step in lambda."""
    xk = fixed_pivot_lslu(op, np.asarray(b, np.float64), k, lam + 1j * h, piv_t, piv_g, x0)
    return float(np.dot(np.asarray(xbar, np.float64), xk.imag) / h)


def vjp_full(op, b, k, lam, piv_t, piv_g, xbar, x0=None):
    """(d x_k / d b)^T xbar, one complex step per entry of b (small m only)."""
    m = op.shape[0]
    out = np.zeros(m)
    for r in range(m):
        e = np.zeros(m)
        e[r] = 1.0
        out[r] = vjp_directional(op, b, k, lam, piv_t, piv_g, xbar, e, x0)
    return out
