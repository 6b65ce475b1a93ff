"""Weak-dangling peeling (PR_PEEL, include/pr.h): IFP2 with the weakly dangling vertices
of section 2 taken out of phase 1 and gathered level by level in phase 2.

Pins: the counts the peeled graph reports against oracle.weak_dangling_levels (pinned
on the CPU in test_oracle_peel.py); results against the FP64 power-method oracle, the
exact closed forms, and the same graph solved without peeling.
Tolerances: L1 <= 1e-9 with FP64 residuals (xi 1e-13), <= 1e-6 with FP32 residuals
under the certified stop.
"""
import numpy as np
import pytest

import oracle
import prgen
from conftest import l1, topk_agree

pytestmark = pytest.mark.gpu
C = 0.85
MAX_LEVELS = 64  # PR_PEEL_MAX_LEVELS


@pytest.fixture(scope="module")
def pr():
    import paper_2302_03245_amd as pr
    pr.lib()
    return pr


def _say(*a):
    print(*a, flush=True)


def _expected_info(g):
    lev = oracle.weak_dangling_levels(g, max_levels=MAX_LEVELS)
    peeled = int((lev >= 1).sum())
    return {"n_peeled": peeled, "peel_levels": int(lev.max()) if peeled else 0,
            "n_dangling": int((lev == 0).sum()), "m_dangling": int((lev[g.col] >= 0).sum()) if g.m else 0}


def _graphs():
    out = [
        ("dag_back", prgen.workload_dag(n_layers=12, layer_size=3000, zmax=200, target_edges=300_000,
                                        back_frac=0.005, seed=2)),
        ("dag_pure", prgen.workload_dag(n_layers=10, layer_size=2000, zmax=100, target_edges=150_000,
                                        back_frac=0.0, seed=4)),
        ("rand_n20011_selfloops_multi", prgen.random_digraph(20011, 150000, seed=2, self_loops=True, multi=True,
                                                            dangling_frac=0.3)),
        ("rand_sparse", prgen.random_digraph(5003, 9000, seed=7, dangling_frac=0.25, unref_frac=0.1)),
        ("rmat_small", prgen.workload_rmat_small(seed=3)),
    ]
    return out


GRAPHS = _graphs()


@pytest.mark.parametrize("name,g", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_peeled_ifp2_matches_oracle(pr, name, g):
    exp = _expected_info(g)
    dg = pr.upload(g.row_ptr, g.col, peel=True)
    info = dg.info()
    _say(f"{name}: n {g.n} m {g.m} peeled {info['n_peeled']} levels {info['peel_levels']}")
    for k, v in exp.items():
        assert info[k] == v, (k, info[k], v)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    plain = pr.upload(g.row_ptr, g.col)
    for mode in (None, "push", "pull", "list"):
        pi, st = pr.ifp2(dg, c=C, xi=1e-13, mode=mode)
        assert st["status"] == 0
        assert l1(pi, ref) <= 1e-9, (mode, l1(pi, ref))
        assert topk_agree(ref, pi, 1000, "fp64")[0]
        pi32, st32 = pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32", mode=mode)
        assert st32["status"] == 0 and st32["l1_bound"] <= 1e-6
        assert l1(pi32, ref) <= 1e-6
        # the reference itself is within c / (1 - c) * 1e-13 of the exact vector
        assert st32["l1_bound"] >= l1(pi32, ref) - 1e-12
    # the sweeps gather fewer edges; phase 2 reads every edge into the deferred vertices once
    # (the threshold stop, whose frontier rule is the same on both graphs: the L1 stop of
    # the plain graph uses the weighted bound, which the peeled graph does not have)
    pi_p, st_p = pr.ifp2(dg, c=C, xi=1e-12)
    pi_n, st_n = pr.ifp2(plain, c=C, xi=1e-12)
    assert l1(pi_p, pi_n) <= 2e-9
    if info["n_peeled"]:
        assert st_p["edges_processed"] < st_n["edges_processed"], (st_p["edges_processed"], st_n["edges_processed"])


def test_chain_beyond_the_level_cap_exact(pr):
    """A chain of 100: the last 65 vertices are dangling or peeled (levels 0..64), the
    first 35 stay in the core; x_k = (1 - c^k) / (1 - c) for the k-th vertex."""
    n = 100
    g = prgen.from_edges(n, np.arange(n - 1), np.arange(1, n))
    dg = pr.upload(g.row_ptr, g.col, peel=True)
    info = dg.info()
    assert info["n_peeled"] == MAX_LEVELS and info["peel_levels"] == MAX_LEVELS
    k = np.arange(1, n + 1)
    y = (1 - C ** k) / (1 - C)
    pi, st = pr.ifp2(dg, c=C, l1_tol=1e-12)
    assert st["status"] == 0 and l1(pi, y / y.sum()) <= 1e-12
    # a chain short enough to peel completely: no core at all
    g = prgen.from_edges(40, np.arange(39), np.arange(1, 40))
    dg = pr.upload(g.row_ptr, g.col, peel=True)
    assert dg.info()["n_peeled"] == 39
    y = (1 - C ** np.arange(1, 41)) / (1 - C)
    pi, st = pr.ifp2(dg, c=C, l1_tol=1e-12)
    assert st["status"] == 0 and st["sweeps"] == 0 and l1(pi, y / y.sum()) <= 1e-12


def test_personalised_ppr_and_literal(pr):
    g = GRAPHS[0][1]
    dg = pr.upload(g.row_ptr, g.col, peel=True)
    lev = oracle.weak_dangling_levels(g, max_levels=MAX_LEVELS)
    p = prgen.random_p(g.n, seed=3, zero_frac=0.5)
    ref_p, _, _ = oracle.power(g, C, p, tol=1e-13)
    pi, st = pr.ifp2(dg, p=p, c=C, xi=1e-13)
    assert l1(pi, ref_p) <= 1e-9
    # sources in the core, at the highest peeled level, at level 1, and dangling
    srcs = [int(np.flatnonzero(lev == -1)[5]), int(np.flatnonzero(lev == lev.max())[0]),
            int(np.flatnonzero(lev == 1)[3]), int(np.flatnonzero(lev == 0)[7])]
    out, stats = pr.ppr(dg, srcs, c=C, xi=1e-13)
    out32, stats32 = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32")
    for r, s in enumerate(srcs):
        e = np.zeros(g.n)
        e[s] = 1.0
        ref, _, _ = oracle.power(g, C, e, tol=1e-13)
        _say(f"ppr source {s} (level {lev[s]}): sweeps {stats[r]['sweeps']}")
        assert stats[r]["status"] == 0 and l1(out[r], ref) <= 1e-9, (s, l1(out[r], ref))
        assert stats32[r]["l1_bound"] <= 1e-6 and l1(out32[r], ref) <= 1e-6
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    pi, st = pr.ifp2(dg, c=C, xi=1e-13, literal=True)
    assert l1(pi, ref) <= 1e-9
    pi, st = pr.ifp2(dg, c=C, xi=1e-6, literal=True)
    assert st["l1_bound"] >= l1(pi, ref)


@pytest.mark.parametrize("shift,groups", [(2, 0), (4, 0), (3, 4)])
def test_tiles_groups_and_tuning(pr, shift, groups):
    g = GRAPHS[0][1]
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col, peel=True, tile_shift=shift, groups=groups)
    assert dg.info()["groups"] == (groups or 1)
    pi, st = pr.ifp2(dg, c=C, xi=1e-13)
    assert st["status"] == 0 and l1(pi, ref) <= 1e-9
    if groups:
        rep = pr.tune(dg, c=C, l1_tol=1e-6, residual="fp32", reps=1)
        _say(f"tune on a peeled graph: {rep}")
        # pr_ppr solves a peeled graph's sources one at a time: the tuner times no batch
        assert rep["batch_ordered"] == -1, rep
        pi, st = pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32")
        assert st["l1_bound"] <= 1e-6 and l1(pi, ref) <= 1e-6


def test_max_sweeps_and_rejections(pr):
    g = GRAPHS[0][1]
    dg = pr.upload(g.row_ptr, g.col, peel=True)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    pi, st = pr.ifp2(dg, c=C, l1_tol=1e-12, max_sweeps=3)
    assert st["status"] == 1 and abs(pi.sum() - 1.0) <= 1e-12
    assert st["l1_bound"] >= l1(pi, ref)
    with pytest.raises(pr.PRError, match="PR_PEEL"):
        pr.ifp1(dg, c=C)
    # the power method runs on the peeled layout (every vertex with out-edges gathers)
    pp, sp_ = pr.power(dg, c=C, l1_tol=1e-11)
    assert sp_["status"] == 0 and l1(pp, ref) <= 1e-9
    pp32, _ = pr.power(dg, c=C, l1_tol=1e-6, residual="fp32")
    assert l1(pp32, ref) <= 1e-6
    st_ = pr.State(g.n)
    with pytest.raises(pr.PRError, match="PR_PEEL"):
        pr.ifp2_warm(dg, st_, c=C)
    srv = pr.Server()
    try:
        with pytest.raises(pr.PRError, match="PR_PEEL"):
            srv.add_graph(dg)
    finally:
        srv.close()
    # still usable afterwards
    pi, st = pr.ifp2(dg, c=C, xi=1e-13)
    assert l1(pi, ref) <= 1e-9


def test_device_input_and_dedupe(pr):
    """Peeling from device buffers (the columns come back to the host for the levels) and
    after collapsing repeated edges; levels against the oracle on the graph the library keeps."""
    import torch
    g = prgen.random_digraph(6000, 15000, seed=31, multi=True, self_loops=True, dangling_frac=0.3)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(torch.tensor(g.row_ptr, device="cuda"), torch.tensor(g.col, device="cuda"), peel=True)
    exp = _expected_info(g)
    info = dg.info()
    assert info["n_peeled"] == exp["n_peeled"] > 0 and info["m_dangling"] == exp["m_dangling"]
    pi, st = pr.ifp2(dg, c=C, xi=1e-13)
    assert st["status"] == 0 and l1(pi, ref) <= 1e-9
    deg = np.diff(g.row_ptr)
    key = np.unique(np.repeat(np.arange(g.n), deg).astype(np.int64) * g.n + g.col)
    gu = prgen.from_edges(g.n, key // g.n, key % g.n)
    dd = pr.upload(g.row_ptr, g.col, dedupe=True, peel=True)
    assert dd.m == gu.m and dd.info()["n_peeled"] == _expected_info(gu)["n_peeled"]
    pi, st = pr.ifp2(dd, c=C, xi=1e-13)
    assert l1(pi, oracle.power(gu, C, tol=1e-13)[0]) <= 1e-9
