"""Pins of oracle.xi_for_l1, the push threshold at which an emptied frontier certifies an
L1 error <= tol (the stop rule of the L1 target: residual left on the non-dangling
vertices at most n_N * xi, unnormalised error at most c / (1 - c) of that, total mass at
least n, normalisation at most doubling the error).  No GPU.

* Tightness: one vertex with a self-loop plus M isolated vertices.  The loop keeps all
  of its mass, so the leftover residual h generates exactly c / (1 - c) * h more mass
  (Eq. 4 on a cycle), and with M large the whole deficit sits on a vertex whose share
  is far from uniform, so normalising doubles it.  With tol placed so that the returned
  threshold sits just above c^k, the oracle's serial IFP2 stops with an error within
  1e-4 of tol, from below; a threshold reaching c^(k-1) stops one pass earlier and
  crosses tol, and each plausible slip in the formula (a dropped 2, c or n / n_N, or
  1 - c on the wrong side) moves the error out of [(1 - 1e-4) tol, tol].  The exact
  vector is the closed form y = (1 / (1 - c), 1, ..., 1).
* Soundness on random graphs (self-loops, repeated edges, dangling and unreferenced
  vertices, personalised p): the serial IFP2 at xi_for_l1(tol) lands within tol of
  the dense exact solve of Eq. 2.
"""
import numpy as np
import pytest

import oracle
import prgen

C = 0.85


def _loop_plus_isolated(M):
    """Vertex 0 with a self-loop, vertices 1..M without edges."""
    n = M + 1
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = 1
    col = np.zeros(1, dtype=np.int32)
    return (n, rp, col)


def _exact_loop(M, c):
    y = np.ones(M + 1)
    y[0] = 1.0 / (1.0 - c)
    return y / y.sum()


def _err_at(xi, M, c):
    g = _loop_plus_isolated(M)
    r = oracle.ifp2(g, c, xi=xi)
    assert r["converged"]
    # the last residual on the loop vertex is a power of c at or below xi
    return float(np.abs(r["pi"] - _exact_loop(M, c)).sum()), r


@pytest.mark.parametrize("k", [30, 45])
def test_xi_for_l1_is_tight_on_a_self_loop(k):
    M = 1_000_000
    n = M + 1
    # tol chosen so that xi_for_l1(tol) sits just above c^k: the loop vertex stops with h = c^k
    tol = 2 * C / (1 - C) * C ** k * (1 + 1e-9) / n
    xi = oracle.xi_for_l1(tol, C, n, 1)
    assert C ** k <= xi < C ** (k - 1)
    err, r = _err_at(xi, M, C)
    assert r["h"][0] == pytest.approx(C ** k, rel=1e-12)
    assert err <= tol
    assert err >= (1 - 1e-4) * tol
    # a threshold reaching c^(k-1) stops one pass earlier and misses the target
    err_hi, _ = _err_at(C ** (k - 1), M, C)
    assert err_hi > tol


def test_xi_for_l1_factor_mistakes_fail():
    """Each plausible slip in the formula moves the stop off the tight case."""
    M, k = 1_000_000, 38
    n = M + 1
    tol = 2 * C / (1 - C) * C ** k * (1 + 1e-9) / n
    good = oracle.xi_for_l1(tol, C, n, 1)
    slips = {
        "dropped 2": tol * (1 - C) / C * n,
        "dropped c": tol * (1 - C) / 2 * n,
        "dropped n / n_N": tol * (1 - C) / (2 * C),
        "1 - c in the denominator": tol * C / (2 * (1 - C)) * n,
    }
    err_good, _ = _err_at(good, M, C)
    assert (1 - 1e-4) * tol <= err_good <= tol
    for name, xi in slips.items():
        err, _ = _err_at(xi, M, C)
        assert not (1 - 1e-4) * tol <= err <= tol, name


GRAPHS = [
    prgen.random_digraph(60, 300, seed=21, dangling_frac=0.2, unref_frac=0.1),
    prgen.random_digraph(40, 220, seed=22, self_loops=True, multi=True, dangling_frac=0.3),
    prgen.random_digraph(80, 160, seed=23, dangling_frac=0.5),
    prgen.workload_dag(n_layers=6, layer_size=12, zmax=8, target_edges=150, back_frac=0.05, seed=6),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("personal", [False, True])
def test_xi_for_l1_is_sound_on_random_graphs(gi, tol, personal):
    g = GRAPHS[gi]
    p = prgen.random_p(g.n, seed=gi + 100, zero_frac=0.3) if personal else None
    n_nd = int((np.diff(g.row_ptr) > 0).sum())
    xi = oracle.xi_for_l1(tol, C, g.n, n_nd)
    r = oracle.ifp2(g, C, p=p, xi=xi)
    assert r["converged"]
    exact = oracle.dense(g, C, p=p, form=0)
    assert float(np.abs(r["pi"] - exact).sum()) <= tol
