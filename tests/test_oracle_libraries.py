"""Oracle against independent library routines (no GPU):
* ``scipy.sparse.linalg.spsolve`` on Eq. 2 with a sparse P' built from the CSR;
* ``networkx.pagerank`` (its default dangling handling follows the
  personalization vector, which is P' = P + p d^T of section 2.1).
"""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import prgen

C = 0.85


def _spsolve_eq2(g, p):
    n = g.n
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(n), deg)
    P = sp.csr_matrix((1.0 / deg[src], (g.col, src)), shape=(n, n))
    dang = (deg == 0).astype(float)
    # (I - cP - c p d^T) pi = (1-c) p ; the rank-one term via Sherman-Morrison
    A = (sp.identity(n, format="csc") - C * P).tocsc()
    u = spla.spsolve(A, p)
    w = spla.spsolve(A, C * p)
    # pi = (1-c) [u + w (d^T u) / (1 - d^T w)]
    return (1 - C) * (u + w * (dang @ u) / (1 - dang @ w))


@pytest.mark.parametrize("seed,n,m", [(1, 200, 1500), (2, 2000, 12000), (3, 6000, 30000)])
def test_power_vs_spsolve(seed, n, m):
    g = prgen.random_digraph(n, m, seed=seed, dangling_frac=0.15, unref_frac=0.1)
    p = prgen.random_p(n, seed) if seed % 2 else np.full(n, 1.0 / n)
    ref = _spsolve_eq2(g, p)
    x, _, _ = oracle.power(g, C, p, tol=1e-14)
    assert np.abs(x - ref).sum() < 1e-11
    r2 = oracle.ifp2(g, C, p, xi=1e-13)
    assert np.abs(r2["pi"] - ref).sum() < 1e-10


def test_power_vs_networkx():
    g = prgen.workload_rmat_small()
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    G.add_edges_from(zip(src.tolist(), g.col.tolist()))
    p = prgen.random_p(g.n, seed=9)
    pr = nx.pagerank(G, alpha=C, personalization={i: p[i] for i in range(g.n)}, tol=1e-15, max_iter=1000)
    ref = np.array([pr[i] for i in range(g.n)])
    x, _, _ = oracle.power(g, C, p, tol=1e-14)
    assert np.abs(x - ref).sum() < 1e-10
