"""Pins of the CPU oracle against exact rational arithmetic (no GPU).

The exact solver (``oracle.exact``) solves the definitions of section 2.1 by
Gauss-Jordan elimination over ``fractions.Fraction``:
* Eq. 2 and Eq. 4 must give the *identical* rational vector (the paper's
  central identity: reserve everything, stop at dangling vertices, normalise
  once);
* that vector must satisfy Eq. 1 exactly (pi = P'' pi, sum 1, positive).
The FP64 oracle routines (dense solve, power method, serial IFP1 / IFP2) must
then land within their own error bounds of the exact answer.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import prgen
from oracle import exact

C = Fraction(17, 20)  # c = 0.85 exactly


def _family():
    """Seeded small digraphs covering self-loops, multi-edges, isolated vertices,
    all-dangling graphs and personalised p (with zeros)."""
    cases = []
    for seed in range(12):
        n = 1 + seed % 7 + (seed // 7)
        m = 3 * n
        g = prgen.random_digraph(n, m, seed=seed, self_loops=seed % 3 == 0, multi=seed % 4 == 1,
                                 dangling_frac=0.25 if seed % 2 else 0.0)
        p = None if seed % 3 else prgen.random_p(n, seed, zero_frac=0.3)
        cases.append((f"rand{seed}", g, p))
    cases.append(("empty3", prgen.from_edges(3, [], []), None))
    cases.append(("single", prgen.from_edges(1, [], []), None))
    cases.append(("selfloop1", prgen.from_edges(1, [0], [0]), None))
    cases.append(("two", prgen.from_edges(2, [0], [1]), None))
    cases.append(("dup", prgen.from_edges(4, [0, 0, 0, 1, 2], [1, 1, 2, 3, 0]), None))
    return cases


CASES = _family()


@pytest.mark.parametrize("name,g,p", CASES, ids=[c[0] for c in CASES])
def test_eq2_equals_eq4_and_eq1(name, g, p):
    pf = None if p is None else [Fraction(float(x)) for x in p]
    a = exact.eq2(g.n, g.row_ptr, g.col, C, pf)
    b = exact.eq4(g.n, g.row_ptr, g.col, C, pf)
    assert a == b, "Eq. 2 and Eq. 4 must give the same rational vector"
    assert sum(a) == 1
    G = exact.google_matrix(g.n, g.row_ptr, g.col, C, pf)
    for i in range(g.n):
        assert sum(G[i][j] * a[j] for j in range(g.n)) == a[i], "pi = P'' pi (Eq. 1)"
    pv = exact._pvec(g.n, pf)
    for i in range(g.n):
        assert a[i] >= (1 - C) * pv[i]
        if pv[i] > 0:
            assert a[i] > 0


@pytest.mark.parametrize("name,g,p", CASES, ids=[c[0] for c in CASES])
def test_oracle_fp64_routines_vs_exact(name, g, p):
    pf = None if p is None else [Fraction(float(x)) for x in p]
    ex = np.array([float(v) for v in exact.eq2(g.n, g.row_ptr, g.col, C, pf)])
    c = 0.85
    for form in (0, 1):
        assert np.abs(oracle.dense(g, c, p, form=form) - ex).sum() <= 1e-14
    x, it, delta = oracle.power(g, c, p, tol=1e-14)
    assert np.abs(x - ex).sum() <= c / (1 - c) * delta + 1e-14
    r1 = oracle.ifp1(g, c, p, xi=1e-15)
    r2 = oracle.ifp2(g, c, p, xi=1e-15)
    assert r1["converged"] and r2["converged"]
    deg = np.diff(g.row_ptr)
    nd = deg > 0
    for r in (r1, r2):
        s_n = r["h"][nd].sum()
        s_x = (r["pibar"] + r["h"]).sum()
        bound = 2 * c / (1 - c) * s_n / max(s_x, 1e-300)
        assert np.abs(r["pi"] - ex).sum() <= bound + 1e-13


def test_literal_ifp2_converges_to_exact():
    """Algorithm 3 read literally (leftover residual dropped) still converges."""
    g = prgen.random_digraph(7, 20, seed=3, dangling_frac=0.3)
    ex = np.array([float(v) for v in exact.eq4(g.n, g.row_ptr, g.col, C)])
    errs = []
    for xi in (1e-3, 1e-6, 1e-9, 1e-12):
        r = oracle.ifp2(g, 0.85, xi=xi, literal=True)
        errs.append(np.abs(r["pi"] - ex).sum())
    assert errs[-1] < 1e-10
    assert errs[0] > errs[-1]


def test_unnormalised_push_target_matches_neumann_series():
    """y = (I - cP)^{-1} h0 equals the truncated series sum_r (cP)^r h0 (Eq. 4's
    algebraic form of forward push) -- checked on a DAG where the series is finite."""
    # 0 -> 1 -> 2, 0 -> 2 : nilpotent P, the series ends after 3 terms
    g = prgen.from_edges(3, [0, 0, 1], [1, 2, 2])
    y = exact.unnormalised(3, g.row_ptr, g.col, C, [1, 1, 1])
    # hand expansion: y0 = 1, y1 = 1 + c/2, y2 = 1 + c/2 + c * y1
    assert y[0] == 1
    assert y[1] == 1 + C / 2
    assert y[2] == 1 + C / 2 + C * (1 + C / 2)
