"""Exact rational PageRank for tiny graphs (test infrastructure only).

Builds P (adjacency normalised by out-degree, multiplicities counted, zero
columns at dangling vertices), d (dangling indicator) and p as
``fractions.Fraction`` matrices, following section 2.1 of the paper, and solves
by Gauss-Jordan elimination in exact arithmetic:

* ``eq2``: (I - c P') pi = (1 - c) p with P' = P + p d^T  (Eq. 2)
* ``eq4``: y = (I - c P)^{-1} p, pi = y / sum(y)          (Eq. 4)
* ``reserve_operator``: R = (I - c P)^{-1}, the operator that maps a residual to
  the mass it will eventually reserve in the 100 %-reserving push.

Pure-Python loops: use only for n of a few dozen at most.
"""
from __future__ import annotations

from fractions import Fraction


def _adjacency(n, row_ptr, col):
    deg = [int(row_ptr[i + 1]) - int(row_ptr[i]) for i in range(n)]
    P = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):
        for e in range(int(row_ptr[j]), int(row_ptr[j + 1])):
            i = int(col[e])
            P[i][j] += Fraction(1, deg[j])
    return P, deg


def _pvec(n, p):
    if p is None:
        return [Fraction(1, n)] * n
    p = [Fraction(x) for x in p]
    s = sum(p)
    return [x / s for x in p]


def _solve(A, b):
    """Gauss-Jordan in exact arithmetic; A is n x n (list of lists), b length n."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for k in range(n):
        piv = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        inv = 1 / M[k][k]
        M[k] = [v * inv for v in M[k]]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k]
                M[r] = [a - f * bk for a, bk in zip(M[r], M[k])]
    return [M[i][n] for i in range(n)]


def eq2(n, row_ptr, col, c, p=None):
    """Exact PageRank from Eq. 2; returns a list of Fractions summing to 1."""
    c = Fraction(c)
    P, deg = _adjacency(n, row_ptr, col)
    pv = _pvec(n, p)
    A = [[(1 if i == j else 0) - c * (P[i][j] + (pv[i] if deg[j] == 0 else 0)) for j in range(n)]
         for i in range(n)]
    return _solve(A, [(1 - c) * x for x in pv])


def eq4(n, row_ptr, col, c, p=None):
    """Exact PageRank from Eq. 4 (solve with P, then normalise once)."""
    c = Fraction(c)
    P, _ = _adjacency(n, row_ptr, col)
    pv = _pvec(n, p)
    A = [[(1 if i == j else 0) - c * P[i][j] for j in range(n)] for i in range(n)]
    y = _solve(A, pv)
    s = sum(y)
    return [v / s for v in y]


def unnormalised(n, row_ptr, col, c, h0):
    """y = (I - c P)^{-1} h0 exactly (the mass a 100 %-reserving push reserves in total)."""
    c = Fraction(c)
    P, _ = _adjacency(n, row_ptr, col)
    A = [[(1 if i == j else 0) - c * P[i][j] for j in range(n)] for i in range(n)]
    return _solve(A, [Fraction(x) for x in h0])


def google_matrix(n, row_ptr, col, c, p=None):
    """P'' = c P' + (1-c) p e^T as exact Fractions (for checking pi = P'' pi, Eq. 1)."""
    c = Fraction(c)
    P, deg = _adjacency(n, row_ptr, col)
    pv = _pvec(n, p)
    return [[c * (P[i][j] + (pv[i] if deg[j] == 0 else 0)) + (1 - c) * pv[i] for j in range(n)]
            for i in range(n)]
