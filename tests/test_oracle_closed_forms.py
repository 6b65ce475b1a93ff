"""Closed-form PageRank vectors (derived by hand from Eq. 4) against every oracle routine.

With uniform p, y = (I - cP)^{-1} e and pi = y / sum(y):
* two vertices 1 -> 2:           pi = (1, 1 + c) / (2 + c)
* chain v1 -> ... -> vn:         y_k = (1 - c^k) / (1 - c)
* out-star centre -> k leaves:   y_centre = 1, y_leaf = 1 + c / k
* in-star k leaves -> centre:    y_leaf = 1, y_centre = 1 + c k
* directed cycle / any graph with all in- and out-degrees equal: pi = e / n
* no edges:                      pi = p
* complete layered DAG (width w, layer l -> l+1): y = (1 - c^(l+1)) / (1 - c)
* PPR from source s on a chain:  y_k = c^(k - s) for k >= s, else 0
"""
import numpy as np
import pytest

import oracle
import prgen

C = 0.85


def _all_routes(g, p=None):
    """pi from every oracle route (power, IFP1, IFP2 folded and literal, dense Eq. 2 / Eq. 4)."""
    out = {}
    out["power"] = oracle.power(g, C, p, tol=1e-15)[0]
    out["ifp1"] = oracle.ifp1(g, C, p, xi=1e-16)["pi"]
    out["ifp2"] = oracle.ifp2(g, C, p, xi=1e-16)["pi"]
    out["ifp2_literal"] = oracle.ifp2(g, C, p, xi=1e-16, literal=True)["pi"]
    if g.n <= 256:
        out["dense2"] = oracle.dense(g, C, p, form=0)
        out["dense4"] = oracle.dense(g, C, p, form=1)
    return out


def _check(g, expect, p=None, tol=1e-12):
    expect = np.asarray(expect, dtype=np.float64)
    for route, pi in _all_routes(g, p).items():
        err = np.abs(pi - expect).sum()
        assert err <= tol, f"{route}: L1 {err:.3e}"


def test_two_vertices():
    g = prgen.from_edges(2, [0], [1])
    expect = np.array([1.0, 1.0 + C]) / (2.0 + C)
    np.testing.assert_allclose(expect, [0.3508771929824561, 0.6491228070175439], rtol=1e-15)
    _check(g, expect)


@pytest.mark.parametrize("n", [2, 5, 40, 300])
def test_chain(n):
    g = prgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    k = np.arange(1, n + 1)
    y = (1 - C ** k) / (1 - C)
    s = (n - C * (1 - C ** n) / (1 - C)) / (1 - C)
    assert abs(y.sum() - s) < 1e-9
    _check(g, y / y.sum())


@pytest.mark.parametrize("k", [1, 3, 17])
def test_out_star(k):
    g = prgen.from_edges(k + 1, np.zeros(k, int), np.arange(1, k + 1))
    expect = np.full(k + 1, (1 + C / k) / (k + 1 + C))
    expect[0] = 1 / (k + 1 + C)
    _check(g, expect)


@pytest.mark.parametrize("k", [1, 4, 33])
def test_in_star(k):
    g = prgen.from_edges(k + 1, np.arange(1, k + 1), np.zeros(k, int))
    expect = np.full(k + 1, 1 / (1 + k + C * k))
    expect[0] = (1 + C * k) / (1 + k + C * k)
    _check(g, expect)


@pytest.mark.parametrize("n", [1, 7, 64])
def test_cycle(n):
    g = prgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    _check(g, np.full(n, 1 / n))


def test_regular_digraph():
    n = 50
    src = np.repeat(np.arange(n), 3)
    dst = (src + np.tile([1, 7, 20], n)) % n
    _check(prgen.from_edges(n, src, dst), np.full(n, 1 / n))


def test_no_edges_gives_p():
    n = 9
    g = prgen.from_edges(n, [], [])
    _check(g, np.full(n, 1 / n))
    p = prgen.random_p(n, seed=4, zero_frac=0.3)
    _check(g, p, p=p)


@pytest.mark.parametrize("layers,w", [(3, 4), (6, 5)])
def test_layered_complete_dag(layers, w):
    n = layers * w
    src, dst = [], []
    for lay in range(layers - 1):
        for a in range(w):
            for b in range(w):
                src.append(lay * w + a)
                dst.append((lay + 1) * w + b)
    g = prgen.from_edges(n, src, dst)
    lay = np.arange(n) // w
    y = (1 - C ** (lay + 1)) / (1 - C)
    _check(g, y / y.sum())


@pytest.mark.parametrize("s", [0, 3])
def test_ppr_chain(s):
    n = 12
    g = prgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    p = np.zeros(n)
    p[s] = 1.0
    k = np.arange(n)
    y = np.where(k >= s, C ** np.clip(k - s, 0, None), 0.0)
    _check(g, y / y.sum(), p=p)
