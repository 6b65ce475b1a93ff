"""Invariants of the 100 %-reserving push (sections 3.1-3.4), checked on the oracle's
intermediate states after a given number of passes.  No GPU.

For a push from a non-dangling vertex i with mass v (pibar_i += v, h_i -= v,
h_j += c v / deg(i) for each target j):
* IFP1 conserves (1 - c) * sum(pibar) + sum(h);
* IFP2 phase 1 (edges into dangling vertices invalidated) conserves
  (1 - c) * sum(pibar) + sum(h) + c * sum_i delta_i * pibar_i, with
  delta_i = (#dangling targets of i) / deg(i);
* at every state, pibar + (I - cP)^{-1} h = (I - cP)^{-1} h0 (IFP1), and the same
  on the non-dangling block with P_NN for IFP2 phase 1.
"""
import numpy as np
import pytest

import oracle
import prgen

C = 0.85


def _dense_P(g):
    n = g.n
    P = np.zeros((n, n))
    deg = np.diff(g.row_ptr)
    for j in range(n):
        for e in range(g.row_ptr[j], g.row_ptr[j + 1]):
            P[g.col[e], j] += 1.0 / deg[j]
    return P, deg


GRAPHS = [
    prgen.random_digraph(60, 300, seed=11, dangling_frac=0.2, unref_frac=0.1),
    prgen.random_digraph(40, 200, seed=12, self_loops=True, multi=True, dangling_frac=0.3),
    prgen.workload_dag(n_layers=6, layer_size=12, zmax=8, target_edges=150, back_frac=0.05, seed=5),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("passes", [1, 2, 3, 7])
def test_ifp1_conservation_and_state_invariant(gi, passes):
    g = GRAPHS[gi]
    r = oracle.ifp1(g, C, xi=1e-14, max_passes=passes)
    h0 = np.ones(g.n)
    cons = (1 - C) * r["pibar"].sum() + r["h"].sum()
    assert abs(cons - h0.sum()) <= 1e-11 * g.n
    P, _ = _dense_P(g)
    R = np.linalg.inv(np.eye(g.n) - C * P)
    y = R @ h0
    np.testing.assert_allclose(r["pibar"] + R @ r["h"], y, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("passes", [1, 2, 5])
def test_ifp2_phase1_conservation_and_state_invariant(gi, passes):
    g = GRAPHS[gi]
    r = oracle.ifp2(g, C, xi=1e-14, max_passes=passes)
    P, deg = _dense_P(g)
    N = deg > 0
    dang_targets = np.zeros(g.n)
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            dang_targets[i] += not N[g.col[e]]
    delta = np.where(N, dang_targets / np.maximum(deg, 1), 0.0)
    cons = (1 - C) * r["pibar"].sum() + r["h"].sum() + C * (delta * r["pibar"]).sum()
    assert abs(cons - g.n) <= 1e-11 * g.n
    # dangling residuals are never touched in phase 1
    np.testing.assert_array_equal(r["h"][~N], 1.0)
    PNN = P[np.ix_(N, N)]
    R = np.linalg.inv(np.eye(N.sum()) - C * PNN)
    np.testing.assert_allclose(r["pibar"][N] + R @ r["h"][N], R @ np.ones(N.sum()), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_ifp2_phase2_is_exact_given_exact_phase1(gi):
    """Phase 2 alone: with phase 1 converged (tiny xi) the dangling block equals
    h0_D + c P_DN y_N exactly (the observation motivating IFP2)."""
    g = GRAPHS[gi]
    r = oracle.ifp2(g, C, xi=1e-16)
    P, deg = _dense_P(g)
    N = deg > 0
    y = np.linalg.solve(np.eye(g.n) - C * P, np.ones(g.n))
    np.testing.assert_allclose(r["x"], y, rtol=1e-12)
    np.testing.assert_allclose(r["x"][~N], 1.0 + C * P[np.ix_(~N, N)] @ y[N], rtol=1e-12)


def test_unreferenced_vertices_bit_identical():
    g = prgen.random_digraph(500, 3000, seed=21, dangling_frac=0.2, unref_frac=0.2)
    indeg = np.bincount(g.col, minlength=g.n)
    U = indeg == 0
    assert U.sum() > 50
    for r in (oracle.ifp1(g, C, xi=1e-12), oracle.ifp2(g, C, xi=1e-12)):
        vals = r["pi"][U]
        assert np.all(vals == vals[0])
        assert np.all(r["pi"][~U] >= vals[0] * (1 - 1e-12))


def test_lower_bound_and_sum():
    g = prgen.workload_rmat_small()
    p = prgen.random_p(g.n, seed=3, zero_frac=0.5)
    for pi in (oracle.power(g, C, p)[0], oracle.ifp1(g, C, p, xi=1e-12)["pi"],
               oracle.ifp2(g, C, p, xi=1e-12)["pi"]):
        assert abs(pi.sum() - 1) < 1e-13
        assert np.all(pi >= (1 - C) * p * (1 - 1e-12))


def test_error_shrinks_with_xi_and_ifp2_saves_pushes():
    """Eq. 8 / Fig. 1 shape: error falls as xi falls; IFP2 performs fewer edge pushes
    than IFP1 at the same xi (the saved pushes into dangling vertices)."""
    g = prgen.workload_rmat_small()
    ref = oracle.power(g, C, tol=1e-14)[0]
    prev = None
    for xi in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        r1 = oracle.ifp1(g, C, xi=xi)
        r2 = oracle.ifp2(g, C, xi=xi)
        e1 = np.abs(r1["pi"] - ref).sum()
        e2 = np.abs(r2["pi"] - ref).sum()
        if prev is not None:
            assert e1 < prev[0] and e2 < prev[1]
        prev = (e1, e2)
        assert r2["edge_pushes"] < r1["edge_pushes"]
        assert r2["vertex_pushes"] <= r1["vertex_pushes"] * 1.05
    assert prev[0] < 1e-8 and prev[1] < 1e-8
