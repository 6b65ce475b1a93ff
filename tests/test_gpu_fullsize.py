"""Parity at the full workload sizes, in the configuration bench.py times.

* R-MAT scale 22 (4,194,304 vertices, 16 * 2^22 draws, 15 % dangling, 10 %
  unreferenced): IFP1 / IFP2 / power with FP32 residuals and the certified
  L1 <= 1e-6 stop, and IFP2 with FP64 residuals at L1 <= 1e-9.
* Layered DAG (2^23 vertices, 64 layers, 80M Zipf edges + 2 % back edges):
  the same FP32 configuration, and IFP2 on the graph uploaded with its weakly
  dangling vertices peeled (counts pinned to oracle.weak_dangling_levels).
Reference: the FP64 power-method oracle over the whole graph (tens of seconds
of one host core).  Every GPU result is compared element by element (L1), by
its top-1000 ranking (tie rule of conftest.topk_agree), and by the
PageRank-equation residual ||pi - cP pi - gamma p||_1, gamma = 1 - c + c d^T pi.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import prgen
from conftest import l1, topk_agree

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
C = 0.85


def _eq_residual(g, pi):
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    inv = np.zeros(g.n)
    inv[deg > 0] = 1.0 / deg[deg > 0]
    P = sp.csr_matrix((inv[src], (g.col, src)), shape=(g.n, g.n))
    gamma = 1 - C + C * pi[deg == 0].sum()
    return float(np.abs(pi - C * (P @ pi) - gamma / g.n).sum())


def _check(pr, g, ref, fp64_too, peel=False):
    dg = pr.upload(g.row_ptr, g.col)
    runs = [("ifp2", lambda: pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32"), 1e-6),
            ("ifp1", lambda: pr.ifp1(dg, c=C, l1_tol=1e-6, residual="fp32"), 1e-6),
            ("power", lambda: pr.power(dg, c=C, l1_tol=1e-6, residual="fp32"), 1e-6)]
    if fp64_too:
        runs.append(("ifp2_fp64", lambda: pr.ifp2(dg, c=C, l1_tol=1e-9), 1e-9))
    if peel:  # weakly dangling vertices out of the sweeps, as the DAG bench line runs it
        dp = pr.upload(g.row_ptr, g.col, peel=True)
        lev = oracle.weak_dangling_levels(g, max_levels=64)
        info = dp.info()
        print(f"{g.name} peeled {info['n_peeled']} in {info['peel_levels']} levels", flush=True)
        assert info["n_peeled"] == int((lev >= 1).sum()) and info["m_dangling"] == int((lev[g.col] >= 0).sum())
        runs.append(("ifp2_peel", lambda: pr.ifp2(dp, c=C, l1_tol=1e-6, residual="fp32"), 1e-6))
    for name, run, tol in runs:
        pi, st = run()
        err = l1(pi, ref)
        ok, swaps, eps = topk_agree(ref, pi, 1000)
        print(f"{g.name} {name}: sweeps {st['sweeps']} L1 {err:.3e} bound {st['l1_bound']:.3e} "
              f"top-1000 swaps {swaps} eps_inf {eps:.2e}", flush=True)
        assert st["status"] == 0 and st["l1_bound"] <= tol
        assert err <= tol
        assert ok
        assert abs(pi.sum() - 1.0) < 1e-10
        assert _eq_residual(g, pi) <= 2 * tol
    dg.free()
    if peel:
        dp.free()


@pytest.mark.timeout(300)
def test_rmat_scale22(pr_lib):
    g = prgen.workload_rmat(scale=22, edge_factor=16, dangling_frac=0.15, unref_frac=0.10, seed=0)
    print(f"R-MAT scale 22: n={g.n} m={g.m}", flush=True)
    ref, it, delta = oracle.power(g, C, tol=1e-13)
    print(f"oracle power: {it} iterations, delta {delta:.2e}", flush=True)
    _check(pr_lib, g, ref, fp64_too=True)


@pytest.mark.timeout(400)
def test_layered_dag(pr_lib):
    g = prgen.workload_dag()
    print(f"layered DAG: n={g.n} m={g.m} lambda={g.meta['lambda']:.4f}", flush=True)
    ref, it, delta = oracle.power(g, C, tol=1e-11)
    print(f"oracle power: {it} iterations, delta {delta:.2e}", flush=True)
    _check(pr_lib, g, ref, fp64_too=False, peel=True)


@pytest.fixture(scope="module")
def pr_lib():
    import paper_2302_03245_amd as pr
    pr.lib()
    return pr


def _eq_residual_c(g, pi, c):
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    inv = np.zeros(g.n)
    inv[deg > 0] = 1.0 / deg[deg > 0]
    P = sp.csr_matrix((inv[src], (g.col, src)), shape=(g.n, g.n))
    gamma = 1 - c + c * pi[deg == 0].sum()
    return float(np.abs(pi - c * (P @ pi) - gamma / g.n).sum())


@pytest.mark.timeout(900)
def test_graph_set_256(pr_lib):
    """The batched workload: 256 R-MAT graphs (n log-uniform in [1k, 500k], average
    degree in [4, 32], 5-20 % dangling, c in {0.85, 0.9}) solved as one set with
    FP32 residuals at L1 <= 1e-6, as bench.py times it.  Every graph: certified
    bound, unit sum, and the PageRank-equation residual within (1 + c) * 1e-6 (it
    holds for any vector within 1e-6 of the solution); the eight smallest graphs
    and two larger ones also against the FP64 oracle element by element."""
    pr = pr_lib
    graphs, cs = prgen.workload_batch(count=256, seed=0)
    print(f"set: n {sum(g.n for g in graphs)} m {sum(g.m for g in graphs)}", flush=True)
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=1e-6, residual="fp32")
    parts = gs.split(pi)
    for i, (g, c, x, st) in enumerate(zip(graphs, cs, parts, sts)):
        assert st["status"] == 0 and st["l1_bound"] <= 1e-6, (i, st)
        assert abs(x.sum() - 1.0) <= 1e-12, i
        r = _eq_residual_c(g, x, c)
        assert r <= (1 + c) * 1e-6, (i, g.n, r)
    order = np.argsort([g.n for g in graphs])
    sample = list(order[:8]) + [int(order[100]), int(order[140])]
    for i in sample:
        ref = oracle.power(graphs[i], cs[i], tol=1e-13)[0]
        d = l1(parts[i], ref)
        print(f"graph {i}: n {graphs[i].n} c {cs[i]} L1 vs oracle {d:.3e}", flush=True)
        assert d <= 1e-6, (i, d)
        ok, swaps, eps = topk_agree(ref, parts[i], min(1000, graphs[i].n))
        assert ok, (i, swaps, eps)
    gs.free()
