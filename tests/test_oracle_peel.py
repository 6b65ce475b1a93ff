"""Pins of oracle.weak_dangling_levels (section 2: deleting the dangling vertices makes
new, weakly dangling ones; the round in which a vertex is deleted is its level).  No GPU.

The levels are checked against closed forms (a chain, a cycle with a tail, a
self-loop) and, on random small graphs, against the property that defines them
uniquely: level 0 exactly for the vertices without out-edges; level L >= 1 when
every out-neighbour has a level in [0, L) and one has level L - 1; -1 (never
deleted) when some out-neighbour is never deleted.
"""
import numpy as np
import pytest

import oracle
import prgen


def test_chain_levels_are_distances_to_the_end():
    n = 50
    g = prgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    assert np.array_equal(oracle.weak_dangling_levels(g), n - 1 - np.arange(n))
    capped = oracle.weak_dangling_levels(g, max_levels=10)
    assert np.array_equal(capped, np.where(n - 1 - np.arange(n) <= 10, n - 1 - np.arange(n), -1))


def test_cycle_with_tail_and_self_loop():
    # 0 -> 1 -> 2 -> 0 (cycle), 2 -> 3 -> 4 (tail, 4 dangling), 5 -> 1 (into the cycle),
    # 6 -> 6 and 6 -> 4 (a self-loop keeps 6), 7 -> 3 and 7 -> 4
    src = [0, 1, 2, 2, 3, 5, 6, 6, 7, 7]
    dst = [1, 2, 0, 3, 4, 1, 6, 4, 3, 4]
    g = prgen.from_edges(8, src, dst)
    assert oracle.weak_dangling_levels(g).tolist() == [-1, -1, -1, 1, 0, -1, -1, 2]


def test_graph_without_edges_and_acyclic_graph():
    assert oracle.weak_dangling_levels(prgen.from_edges(4, [], [])).tolist() == [0, 0, 0, 0]
    # a DAG peels completely
    g = prgen.workload_dag(n_layers=6, layer_size=20, zmax=8, target_edges=300, back_frac=0.0, seed=3)
    lev = oracle.weak_dangling_levels(g)
    assert (lev >= 0).all()


def _check_defining_property(g, lev):
    deg = np.diff(g.row_ptr)
    for v in range(g.n):
        outs = lev[g.col[g.row_ptr[v]:g.row_ptr[v + 1]]]
        if deg[v] == 0:
            assert lev[v] == 0
        elif lev[v] >= 1:
            assert (outs >= 0).all() and (outs < lev[v]).all() and outs.max() == lev[v] - 1
        else:
            assert lev[v] == -1 and (outs == -1).any()


@pytest.mark.parametrize("seed", range(12))
def test_defining_property_on_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 60))
    m = int(rng.integers(0, 3 * n))
    # mostly forward edges so that long peel chains occur, some backward ones close cycles
    src = rng.integers(0, n, m)
    dst = np.where(rng.random(m) < 0.9, np.minimum(src + rng.integers(0, 4, m), n - 1), rng.integers(0, n, m))
    keep = rng.random(n) < 0.15
    g = prgen.from_edges(n, src[~keep[src]], dst[~keep[src]])
    lev = oracle.weak_dangling_levels(g)
    _check_defining_property(g, lev)
    for cap in (0, 1, 3):
        capped = oracle.weak_dangling_levels(g, max_levels=cap)
        assert np.array_equal(capped, np.where(lev <= cap, lev, -1))
