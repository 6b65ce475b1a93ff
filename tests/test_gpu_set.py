"""Graph sets (include/pr_set.h): many independent graphs solved in one set of launches.

Every graph's result is checked against the FP64 oracle (power method to
1e-13) within the certified tolerance, against the same graph solved alone
through pr_solve_ifp2, and for the closed forms against the exact vector.
Synchronous set sweeps follow each graph's solo synchronous trajectory (same
sweep count up to one); ordered set sweeps (vertex groups per graph, the
default) are checked against the oracle and need no more sweeps in total.
Tolerances: L1 <= 1e-9 with FP64 residuals, L1 <= 1e-6 with FP32 residuals.
"""
import numpy as np
import pytest

import oracle
import prgen
from conftest import l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import paper_2302_03245_amd as pr
    pr.lib()
    return pr


def _say(*a):
    print(*a, flush=True)


def _mixed_graphs():
    """Uneven sizes, empty and all-dangling graphs, hubs, mixed damping factors."""
    gs = [
        prgen.from_edges(1, [], []),
        prgen.from_edges(1, [0], [0]),
        prgen.from_edges(5, [], []),
        prgen.from_edges(2, [0], [1]),
        prgen.from_edges(37, np.arange(36), np.arange(1, 37)),
        prgen.from_edges(5001, np.zeros(5000, int), np.arange(1, 5001)),
        prgen.from_edges(5001, np.arange(1, 5001), np.zeros(5000, int)),
        prgen.workload_rmat_small(seed=0),
    ]
    for i, (n, m, dfr) in enumerate([(3, 6, 0.0), (50, 300, 0.2), (300, 2500, 0.1), (2000, 16000, 0.3),
                                     (20011, 150000, 0.15), (777, 777, 0.5), (4096, 70000, 0.05)]):
        gs.append(prgen.random_digraph(n, m, seed=40 + i, dangling_frac=dfr, unref_frac=0.1))
    for i in range(6):
        gs.append(prgen.workload_rmat_n(int(1000 * 3 ** i) + 17 * i, 4 + 5 * i, 0.05 + 0.03 * i, seed=90 + i))
    rng = np.random.default_rng(3)
    cs = rng.choice([0.85, 0.9], len(gs))
    cs[0], cs[-1] = 0.5, 0.99
    return gs, [float(x) for x in cs]


_ORACLE = {}


def _oracle(g, c, key):
    if key not in _ORACLE:
        _ORACLE[key] = oracle.power(g, c, tol=1e-13)[0]
    return _ORACLE[key]


@pytest.mark.parametrize("residual,tol,mode", [("fp64", 1e-9, None), ("fp32", 1e-6, None),
                                               ("fp64", 1e-9, "push"), ("fp32", 1e-6, "pull")])
def test_set_matches_oracle_and_alone(pr, residual, tol, mode):
    graphs, cs = _mixed_graphs()
    _say(f"set of {len(graphs)} graphs, n = {sum(g.n for g in graphs)}, residual {residual}, mode {mode}")
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs], groups=1)
    assert gs.info()["groups"] == 1
    pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=tol, residual=residual, mode=mode)
    for i, (g, c, x, st) in enumerate(zip(graphs, cs, gs.split(pi), sts)):
        assert st["status"] == 0, (i, st)
        assert st["l1_bound"] <= tol, (i, st)
        assert abs(x.sum() - 1.0) <= 1e-12, i
        ref = _oracle(g, c, (i, c))
        assert l1(x, ref) <= tol, (i, g.n, c, l1(x, ref))
        dg = pr.upload(g.row_ptr, g.col)
        alone, sa = pr.ifp2(dg, c=c, l1_tol=tol, residual=residual, mode=mode, jacobi=True)
        assert l1(x, alone) <= 2 * tol, (i, l1(x, alone))
        # same Jacobi trajectory per graph, only the rounding order differs; the solo
        # solve's stop rule weighs each vertex's residual by its own error weight, never
        # above the set's uniform c / (1 - c), so it stops no later
        assert sa["sweeps"] <= st["sweeps"] + 1, (i, st["sweeps"], sa["sweeps"])


@pytest.mark.parametrize("residual,tol,groups", [("fp64", 1e-9, 0), ("fp32", 1e-6, 0), ("fp64", 1e-9, 3),
                                                 ("fp32", 1e-6, 15)])
def test_ordered_set_sweeps(pr, residual, tol, groups):
    """Ordered sweeps over per-graph vertex groups: every graph against the oracle and
    against its solo solve; no more sweeps in total than synchronous set sweeps."""
    graphs, cs = _mixed_graphs()
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs], groups=groups)
    assert gs.info()["groups"] == (groups or 4)
    pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=tol, residual=residual)
    _, sync = pr.set_ifp2(gs, c=cs, l1_tol=tol, residual=residual, jacobi=True)
    tot_o, tot_s = sum(st["sweeps"] for st in sts), sum(st["sweeps"] for st in sync)
    _say(f"groups {groups or 4}: sweeps ordered {tot_o} synchronous {tot_s}")
    assert tot_o <= tot_s
    for i, (g, c, x, st) in enumerate(zip(graphs, cs, gs.split(pi), sts)):
        assert st["status"] == 0 and st["l1_bound"] <= tol, (i, st)
        assert abs(x.sum() - 1.0) <= 1e-12, i
        ref = _oracle(g, c, (i, c))
        assert l1(x, ref) <= tol, (i, g.n, c, l1(x, ref))
        if residual == "fp64":  # the bound holds in exact arithmetic; FP32 weights round at ~1e-8
            assert st["l1_bound"] >= l1(x, ref) - 1e-12, i
        alone, _ = pr.ifp2(pr.upload(g.row_ptr, g.col, groups=groups or 4), c=c, l1_tol=tol, residual=residual)
        assert l1(x, alone) <= 2 * tol, (i, l1(x, alone))


def test_set_closed_forms_exact(pr):
    c = 0.85
    n = 37
    k = np.arange(1, n + 1)
    y = (1 - c ** k) / (1 - c)
    chain = (prgen.from_edges(n, np.arange(n - 1), np.arange(1, n)), y / y.sum())
    kk = 40
    e = np.full(kk + 1, 1 / (1 + kk + c * kk))
    e[0] = (1 + c * kk) / (1 + kk + c * kk)
    in_star = (prgen.from_edges(kk + 1, np.arange(1, kk + 1), np.zeros(kk, int)), e)
    cyc = (prgen.from_edges(100, np.arange(100), (np.arange(100) + 1) % 100), np.full(100, 0.01))
    cases = [chain, in_star, cyc, chain]
    gs = pr.upload_set([(g.row_ptr, g.col) for g, _ in cases])
    pi, sts = pr.set_ifp2(gs, c=c, l1_tol=1e-12, residual="fp64")
    for (g, exact), x, st in zip(cases, gs.split(pi), sts):
        assert st["status"] == 0
        assert l1(x, exact) <= 1e-12


def test_many_tiny_graphs(pr):
    """More graphs than one workgroup keeps in LDS: per-graph sums go through device atomics."""
    rng = np.random.default_rng(8)
    graphs = []
    for i in range(300):
        n = int(rng.integers(1, 41))
        graphs.append(prgen.random_digraph(n, int(rng.integers(0, 4 * n + 1)), seed=1000 + i,
                                           dangling_frac=float(rng.uniform(0, 0.4))))
    cs = [0.85 if i % 3 else 0.9 for i in range(len(graphs))]
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=1e-10, residual="fp64")
    for i, (g, c, x, st) in enumerate(zip(graphs, cs, gs.split(pi), sts)):
        assert st["status"] == 0 and st["l1_bound"] <= 1e-10
        ref = oracle.dense(g, c) if g.n <= 12 else oracle.power(g, c, tol=1e-13)[0]
        assert l1(x, ref) <= 1e-10, (i, g.n, l1(x, ref))


def test_set_xi_rule_and_device_output(pr):
    import torch
    graphs, _ = _mixed_graphs()
    graphs = graphs[4:12]
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    out = torch.empty(gs.n, dtype=torch.float64, device="cuda")
    pi, sts = pr.set_ifp2(gs, c=0.85, xi=1e-11, residual="fp64", out=out, jacobi=True)
    got = gs.split(out.cpu().numpy())
    for g, x, st in zip(graphs, got, sts):
        dg = pr.upload(g.row_ptr, g.col)
        alone, sa = pr.ifp2(dg, c=0.85, xi=1e-11, residual="fp64", jacobi=True)
        assert l1(x, alone) <= 1e-12
        assert abs(st["sweeps"] - sa["sweeps"]) <= 1


def test_set_max_sweeps_and_rejections(pr):
    graphs, cs = _mixed_graphs()
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=1e-9, residual="fp64", max_sweeps=3)
    assert sts[0]["status"] == 1  # PR_ENOCONV for the set
    assert any(st["l1_bound"] > 1e-9 for st in sts)
    for x in gs.split(pi):
        assert abs(x.sum() - 1.0) <= 1e-12   # normalised best estimate
    with pytest.raises(pr.PRError, match="every c"):
        pr.set_ifp2(gs, c=[1.5] * gs.k, l1_tol=1e-6)
    with pytest.raises(ValueError):
        pr.set_ifp2(gs, c=[0.85] * (gs.k + 1), l1_tol=1e-6)


def test_set_tune_keeps_results(pr):
    """The set autotuner times every tile size with synchronous and ordered sweeps and
    keeps the fastest; results stay within the tolerance afterwards."""
    graphs, cs = _mixed_graphs()
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    rep = pr.set_tune(gs, c=cs, l1_tol=1e-6, residual="fp32", reps=1)
    _say(f"set tune: {rep}")
    assert len(rep["candidates"]) == 6
    assert {(x["tile_shift"], x["ordered"]) for x in rep["candidates"]} == {(s, o) for s in (2, 3, 4)
                                                                           for o in (False, True)}
    info = gs.info()
    assert info["tile_items"] == 256 << rep["chosen"]["tile_shift"]
    assert bool(info["ordered"]) == rep["chosen"]["ordered"]
    for residual, tol in (("fp32", 1e-6), ("fp64", 1e-9)):
        pi, sts = pr.set_ifp2(gs, c=cs, l1_tol=tol, residual=residual)
        for i, (g, c, x, st) in enumerate(zip(graphs, cs, gs.split(pi), sts)):
            assert st["status"] == 0 and st["l1_bound"] <= tol
            assert l1(x, _oracle(g, c, (i, c))) <= tol, i
    with pytest.raises(pr.PRError, match="automatic schedule"):
        o = pr._opts(0.85, 1e-12, 1e-6, "fp32", 0, None, False, "push", False)
        r = pr.TuneReport()
        st = pr.lib().pr_set_tune(gs.handle, None, o, 1, r)
        raise pr._err(st)
