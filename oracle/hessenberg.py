"""Algorithm 5 (Hybrid LSLU) with Algorithm 4's pivoting, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each iteration of Algorithm 5 is built from the same two steps on both
bases (``eliminate``: the components along the earlier basis vectors, each
read at that vector's pivot row and removed in turn; ``take_pivot``: the
infinity-norm pivot, the division by it and the update of the permutation),
in the paper's notation: permutation vectors ``t`` (rows, for the basis ``D``)
and ``g`` (columns, for the basis ``L``), the adjoint product
``q = A^T d_k`` reduced against ``L``, the forward product ``u = A l_k``
reduced against ``D``, then the choice of lambda_k, the projected Tikhonov
solve and the iterate ``x_k = x_0 + L_k y``.  Elimination is sequential in j,
as the method defines it; the relations ``A L_k = D_{k+1} H_{k+1,k}`` and
``A^T D_k = L_k W_k`` that these steps build are pinned by the tests.

Readings where the paper is silent, ambiguous or inconsistent:

* R1 (guard of the l_k pivot): the paper writes ``k < n`` but searches
  ``i in {k..n}``.  The guard used is ``k <= n`` (search range non-empty), so a
  square system can reach full dimension.  The d_{k+1} guard ``k < m`` is used
  as written.
* R2 (what happens at a breakdown): Algorithm 5 breaks out of the loop before
  lambda/y/x.  On the u side (``u = 0`` or ``k >= m``) the oracle follows
  Algorithm 2 instead: ``H(k+1,k) = 0``, then ``x_k`` is still formed and the
  loop stops.  On the q side the loop stops and the result is ``x_{k-1}``
  (``x_0`` when ``k = 1``).
* R3 (``q != 0``, ``u != 0``): exact test, i.e. the largest magnitude over the
  entries still eligible as pivots is exactly zero.
* R4 (ties in the pivot search): the smallest vector index among the entries of
  largest magnitude; only entries not yet used as pivots are eligible.
* R6 (normalisation): IEEE division by the pivot value, so the pivot entry is
  exactly 1 and every entry has magnitude at most 1.
* R7 (beta): the signed entry ``r_0(i)``.
* R8 (regularisation term): the penalty is on ``y``, i.e. on
  ``L_k^+ (x - x_0)``; this matches eq. TP when ``x_0 = 0``.
* R19 (sampled pivots, the variant proposed in Section 2.2 and shown in
  Fig. 1): the paper does not say how the sample is drawn.  Each search gets
  a list of distinct random rows of its vector (an input, from
  ``workloads.pivot_sample_lists``); the sample is the first s rows of that
  list that are not earlier pivots (so s non-pivot rows, without
  replacement), the pivot is the sampled row of largest magnitude (ties:
  smallest row), and a sample whose largest magnitude is 0 falls back to the
  full search, so breakdown is still decided exactly (R3).
* R13 (stopping): ``k_stop`` is the first ``k`` with
  ``|Ghat(k+1) - Ghat(k)| / Ghat(1) < tol``; it is reported and only ends the
  loop when ``early_stop`` is set (then the result is ``x_{k_stop}``).
"""

from __future__ import annotations

import dataclasses
import enum
from typing import List, Optional

import numpy as np

from .projected import (RegParam, ghat_value, projected_svd, select_lambda,
                        tikhonov_coeffs)


class Status(enum.IntEnum):
    OK = 0
    BREAKDOWN_Q = 1
    BREAKDOWN_U = 2
    ZERO_RHS = 3


@dataclasses.dataclass
class Result:
    status: Status
    k_done: int  # number of iterates x_1..x_k formed
    x: np.ndarray  # final iterate (x_{k_done}, or x_{k_stop} with early_stop)
    beta: float
    piv_t: List[int]  # t(1), t(2), ... : row pivots of d_1, d_2, ...
    piv_g: List[int]  # g(1), g(2), ... : column pivots of l_1, l_2, ...
    H: np.ndarray  # (K+1) x K
    W: np.ndarray  # K x K
    L: np.ndarray  # n x (number of l's formed)
    D: np.ndarray  # m x (number of d's formed)
    X: np.ndarray  # n x k_done, column k-1 is x_k
    Y: np.ndarray  # K x K, column k-1 holds y_k in rows 0..k-1
    lambdas: np.ndarray  # lambda_k, k = 1..k_done
    lambda_idx: np.ndarray  # grid index of lambda_k (-1 if no grid)
    ghat: np.ndarray  # Ghat(k), k = 1..k_done
    sep_t: List[float]  # pivot separation at each d-side search (incl. r_0)
    sep_g: List[float]  # pivot separation at each l-side search
    sep_lambda: np.ndarray  # grid separation of lambda_k
    k_stop: int


def pivot_search(v: np.ndarray, perm: np.ndarray, start: int):
    """Algorithm 4's "determine i in {start..} such that |v(perm(i))| is the
    infinity norm of v(perm(start:))" with reading R4 for ties.

    Returns ``(pos, amax, sep)``: the position in ``perm`` (0-based), the
    largest magnitude, and the separation ``(a1 - a2)/a1`` between the largest
    and second largest magnitudes among the candidates (1 if there is one
    candidate, 0 if the largest is 0)."""
    cand = perm[start:]
    a = np.abs(v[cand])
    amax = a.max()
    hits = np.nonzero(a == amax)[0]
    pos = start + int(hits[np.argmin(cand[hits])])
    if amax == 0:
        sep = 0.0
    elif a.shape[0] == 1:
        sep = 1.0
    else:
        a2 = np.partition(a, a.shape[0] - 2)[a.shape[0] - 2]
        sep = float((amax - a2) / amax)
    return pos, float(amax), sep


def pivot_search_sampled(v: np.ndarray, perm: np.ndarray, start: int,
                         cand_rows: np.ndarray, s: int):
    """The sampled pivot of Section 2.2 (reading R19): among the first s rows
    of ``cand_rows`` that are not earlier pivots (``perm[:start]``), the row
    of largest |v| (ties: smallest row).  Falls back to ``pivot_search`` when
    that largest magnitude is 0.  Same return values as ``pivot_search``."""
    used = np.zeros(v.shape[0], dtype=bool)
    used[perm[:start]] = True
    sel = [int(r) for r in cand_rows if r >= 0 and not used[r]][:s]
    a = np.abs(v[sel]) if sel else np.zeros(0)
    if a.shape[0] == 0 or a.max() == 0.0:
        return pivot_search(v, perm, start)
    amax = a.max()
    row = min(r for r, ar in zip(sel, a) if ar == amax)
    pos = int(np.nonzero(perm == row)[0][0])
    if a.shape[0] == 1:
        sep = 1.0
    else:
        a2 = np.partition(a, a.shape[0] - 2)[a.shape[0] - 2]
        sep = float((amax - a2) / amax)
    return pos, float(amax), sep


def eliminate(v: np.ndarray, basis, perm: np.ndarray, count: int, coef: np.ndarray):
    """Removes from ``v`` its components along the first ``count`` basis
    vectors, each measured at that vector's own pivot row: for j = 0, 1, ...,
    count-1 in turn, ``coef[j] = v(perm[j])`` and ``v <- v - coef[j] basis[j]``
    (the inner loops of Algorithm 5 for both bases, of Algorithm 2 for its one
    basis).  Basis vector j is 1 at ``perm[j]`` and 0 at ``perm[:j]``, so the
    result is 0 at ``perm[:count]``.  ``coef`` is written in place (a column
    of W or H).  Returns the new vector."""
    for j in range(count):
        coef[j] = v[perm[j]]
        v = v - coef[j] * basis[j]
    return v


def take_pivot(v: np.ndarray, perm: np.ndarray, start: int, pos: int):
    """Accepts the pivot found at position ``pos`` of ``perm``: returns its
    value ``v(perm[pos])`` and ``v`` divided by it (IEEE division, reading R6:
    exactly 1 at the pivot), and moves the pivot row to position ``start`` of
    ``perm`` (in place)."""
    val = v[perm[pos]]
    perm[start], perm[pos] = perm[pos], perm[start]
    return val, v / val


def hybrid_lslu(op, b, maxiter: int, reg: Optional[RegParam] = None,
                x0: Optional[np.ndarray] = None, stop_tol: float = 1e-6,
                early_stop: bool = False, pivot_sample=None) -> Result:
    """Hybrid LSLU (Algorithm 5); ``reg=None`` or ``RegParam('none')`` gives
    LSLU (lambda = 0).  ``pivot_sample = (lists, s)`` selects the sampled
    pivots of Section 2.2 (reading R19): ``lists[i]`` holds the candidate
    rows of search i (0: r_0; 2k-1: q of iteration k; 2k: u of iteration
    k)."""
    reg = reg if reg is not None else RegParam("none")
    m, n = op.shape
    K = int(maxiter)
    b = np.asarray(b, dtype=np.float64)
    x0v = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)

    t = np.arange(m)
    g = np.arange(n)
    H = np.zeros((K + 1, K))
    W = np.zeros((K, K))
    Y = np.zeros((K, K))
    Lb: List[np.ndarray] = []
    Db: List[np.ndarray] = []
    X: List[np.ndarray] = []
    lambdas, lam_idx, ghat, sep_lam = [], [], [], []
    sep_t: List[float] = []
    sep_g: List[float] = []

    def finish(status, x_final, k_stop):
        kd = len(X)
        return Result(
            status=status, k_done=kd, x=x_final, beta=beta,
            piv_t=[int(v) for v in t[:len(Db)]],
            piv_g=[int(v) for v in g[:len(Lb)]],
            H=H, W=W,
            L=np.stack(Lb, axis=1) if Lb else np.zeros((n, 0)),
            D=np.stack(Db, axis=1) if Db else np.zeros((m, 0)),
            X=np.stack(X, axis=1) if X else np.zeros((n, 0)),
            Y=Y, lambdas=np.array(lambdas), lambda_idx=np.array(lam_idx),
            ghat=np.array(ghat), sep_t=sep_t, sep_g=sep_g,
            sep_lambda=np.array(sep_lam), k_stop=k_stop)

    def search(v, perm, start, i):
        if pivot_sample is None:
            return pivot_search(v, perm, start)
        lists, s = pivot_sample
        return pivot_search_sampled(v, perm, start, lists[i], s)

    # r_0 = b - A x_0; the pivot of r_0; beta; d_1.
    r0 = b - op.matvec(x0v) if x0 is not None else b.copy()
    pos, amax, sep = search(r0, t, 0, 0)
    beta = 0.0
    if amax == 0.0:
        return finish(Status.ZERO_RHS, x0v.copy(), 0)
    sep_t.append(sep)
    beta, d1 = take_pivot(r0, t, 0, pos)
    beta = float(beta)
    Db.append(d1)

    status = Status.OK
    k_stop = None
    x_final = x0v.copy()
    for k in range(1, K + 1):
        # Adjoint product and elimination of l_1..l_{k-1}.
        q = eliminate(op.rmatvec(Db[k - 1]), Lb, g, k - 1, W[:, k - 1])
        # Pivot for l_k (guard k <= n, reading R1; exact zero test, R3).
        if k <= n:
            pos, amax, sep = search(q, g, k - 1, 2 * k - 1)
        else:
            amax = 0.0
        if amax == 0.0:
            status = Status.BREAKDOWN_Q
            break
        sep_g.append(sep)
        W[k - 1, k - 1], lk = take_pivot(q, g, k - 1, pos)
        Lb.append(lk)

        # Forward product and elimination of d_1..d_k.
        u = eliminate(op.matvec(Lb[k - 1]), Db, t, k, H[:, k - 1])
        last = False
        if k < m:
            pos, amax, sep = search(u, t, k, 2 * k)
        else:
            amax = 0.0
        if amax == 0.0:
            H[k, k - 1] = 0.0
            status = Status.BREAKDOWN_U
            last = True
        else:
            sep_t.append(sep)
            H[k, k - 1], dk = take_pivot(u, t, k, pos)
            Db.append(dk)

        # Projected problem: lambda_k, y_k, x_k.
        Hk = H[:k + 1, :k]
        s, c, V = projected_svd(Hk)
        Lk = np.stack(Lb, axis=1)
        lam, li, sl, _ = select_lambda(reg, k, m, beta, s, c, V, Lk, x0v)
        y = tikhonov_coeffs(beta, s, c, V, lam)
        Y[:k, k - 1] = y
        xk = x0v + Lk @ y
        X.append(xk)
        x_final = xk
        lambdas.append(lam)
        lam_idx.append(li)
        sep_lam.append(sl)
        ghat.append(ghat_value(k, n, m, beta, s, c, lam))

        # Stopping rule (eq. tol): decided once Ghat(k) and Ghat(k-1) exist.
        if k_stop is None and k >= 2 and ghat[0] != 0.0:
            if abs(ghat[k - 1] - ghat[k - 2]) / ghat[0] < stop_tol:
                k_stop = k - 1
                if early_stop:
                    x_final = X[k_stop - 1]
                    res = finish(status, x_final, k_stop)
                    return res
        if last:
            break

    kd = len(X)
    return finish(status, x_final, k_stop if k_stop is not None else kd)


def square_hessenberg_pivoted(apply_B, r0: np.ndarray, maxiter: int):
    """Algorithm 2 (Hessenberg process with pivoting) for a square operator
    ``B``: returns ``(Lbasis, Hess, p)`` with ``B L_k = L_{k+1} Hess_{k+1,k}``
    (eq. Hess1) and ``p`` the pivot rows in order.  Same tie rule (R4)."""
    r0 = np.asarray(r0, dtype=np.float64)
    N = r0.shape[0]
    p = np.arange(N)
    pos, amax, _ = pivot_search(r0, p, 0)
    if amax == 0.0:
        raise ValueError("zero start vector")
    beta, l1 = take_pivot(r0, p, 0, pos)
    Lb = [l1]
    Hs = np.zeros((maxiter + 1, maxiter))
    kk = 0
    for k in range(1, maxiter + 1):
        u = eliminate(apply_B(Lb[k - 1]), Lb, p, k, Hs[:, k - 1])
        kk = k
        if k < N:
            pos, amax, _ = pivot_search(u, p, k)
        else:
            amax = 0.0
        if amax == 0.0:
            Hs[k, k - 1] = 0.0
            break
        Hs[k, k - 1], lk = take_pivot(u, p, k, pos)
        Lb.append(lk)
    return np.stack(Lb, axis=1), Hs[:kk + 1, :kk], [int(v) for v in p[:len(Lb)]]
