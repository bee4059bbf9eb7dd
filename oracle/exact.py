"""LSLU (Algorithm 5 with lambda = 0) in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Same steps, order and readings (R1-R4, R6, R7) as ``hessenberg.hybrid_lslu``,
with every number a ``fractions.Fraction``.  The projected least-squares
problem ``min ||beta e_1 - H y||`` (Section 2.2) is solved exactly through its
normal equations ``H^T H y = beta H^T e_1`` by Gaussian elimination, which is
exact in rationals whenever ``H`` has full column rank.  Intended for tiny
integer problems: exact breakdowns (rank deficiency) and exact solution at full
dimension can only be observed here.
"""

from __future__ import annotations

from fractions import Fraction
from typing import List

from .hessenberg import Status


def _matvec(A, x):
    return [sum((a * b for a, b in zip(row, x)), Fraction(0)) for row in A]


def _rmatvec(A, y):
    n = len(A[0])
    out = [Fraction(0)] * n
    for i, row in enumerate(A):
        yi = y[i]
        if yi != 0:
            for j in range(n):
                out[j] += row[j] * yi
    return out


def _search(v, perm, start):
    best_pos, best = None, Fraction(-1)
    for pos in range(start, len(perm)):
        a = abs(v[perm[pos]])
        if a > best or (a == best and perm[pos] < perm[best_pos]):
            best, best_pos = a, pos
    return best_pos, best


def _solve_spd(M, r):
    """Gaussian elimination (no pivoting needed for SPD, exact in Q)."""
    k = len(r)
    M = [row[:] + [r[i]] for i, row in enumerate(M)]
    for c in range(k):
        piv = M[c][c]
        if piv == 0:
            raise ZeroDivisionError("singular projected normal equations")
        for rr in range(c + 1, k):
            f = M[rr][c] / piv
            if f != 0:
                for cc in range(c, k + 1):
                    M[rr][cc] -= f * M[c][cc]
    y = [Fraction(0)] * k
    for c in range(k - 1, -1, -1):
        s = M[c][k] - sum((M[c][j] * y[j] for j in range(c + 1, k)), Fraction(0))
        y[c] = s / M[c][c]
    return y


def hybrid_lslu_exact(A_int, b_int, maxiter: int):
    """LSLU in rationals.  ``A_int``: list of rows (ints or Fractions)."""
    A = [[Fraction(v) for v in row] for row in A_int]
    b = [Fraction(v) for v in b_int]
    m, n = len(A), len(A[0])
    t = list(range(m))
    g = list(range(n))
    K = maxiter
    H = [[Fraction(0)] * K for _ in range(K + 1)]
    W = [[Fraction(0)] * K for _ in range(K)]
    Lb: List[list] = []
    Db: List[list] = []
    X: List[list] = []
    r0 = b[:]
    pos, amax = _search(r0, t, 0)
    if amax == 0:
        return dict(status=Status.ZERO_RHS, k_done=0, x=[Fraction(0)] * n,
                    piv_t=[], piv_g=[], H=H, W=W, L=Lb, D=Db, X=X, beta=0)
    beta = r0[t[pos]]
    Db.append([v / beta for v in r0])
    t[0], t[pos] = t[pos], t[0]
    status = Status.OK
    x = [Fraction(0)] * n
    for k in range(1, K + 1):
        q = _rmatvec(A, Db[k - 1])
        for j in range(1, k):
            W[j - 1][k - 1] = q[g[j - 1]]
            q = [qi - W[j - 1][k - 1] * li for qi, li in zip(q, Lb[j - 1])]
        if k <= n:
            pos, amax = _search(q, g, k - 1)
        else:
            amax = 0
        if amax == 0:
            status = Status.BREAKDOWN_Q
            break
        W[k - 1][k - 1] = q[g[pos]]
        Lb.append([qi / W[k - 1][k - 1] for qi in q])
        g[k - 1], g[pos] = g[pos], g[k - 1]
        u = _matvec(A, Lb[k - 1])
        for j in range(1, k + 1):
            H[j - 1][k - 1] = u[t[j - 1]]
            u = [ui - H[j - 1][k - 1] * di for ui, di in zip(u, Db[j - 1])]
        last = False
        if k < m:
            pos, amax = _search(u, t, k)
        else:
            amax = 0
        if amax == 0:
            H[k][k - 1] = Fraction(0)
            status = Status.BREAKDOWN_U
            last = True
        else:
            H[k][k - 1] = u[t[pos]]
            Db.append([ui / H[k][k - 1] for ui in u])
            t[k], t[pos] = t[pos], t[k]
        # min ||beta e1 - H_{k+1,k} y|| via the normal equations.
        Hk = [row[:k] for row in H[:k + 1]]
        M = [[sum((Hk[r][i] * Hk[r][j] for r in range(k + 1)), Fraction(0))
              for j in range(k)] for i in range(k)]
        rhs = [beta * Hk[0][i] for i in range(k)]
        y = _solve_spd(M, rhs)
        x = [sum((Lb[j][r] * y[j] for j in range(k)), Fraction(0))
             for r in range(n)]
        X.append(x)
        if last:
            break
    return dict(status=status, k_done=len(X), x=x, beta=beta,
                piv_t=t[:len(Db)], piv_g=g[:len(Lb)], H=H, W=W, L=Lb, D=Db,
                X=X)
