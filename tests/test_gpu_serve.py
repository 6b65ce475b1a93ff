"""The query server (include/pr_serve.h): every result is the same alone and in the mix.

Queries (global PageRank and single-source PPR) on two resident graphs arrive in
waves while earlier ones are still on the device; each result is compared with
the same query solved alone through pr_ppr / pr_solve_ifp2 and with the FP64
oracle, within the certified tolerance.
"""
import time

import numpy as np
import pytest

import oracle
import prgen
from conftest import l1

pytestmark = pytest.mark.gpu
C = 0.85


@pytest.fixture(scope="module")
def pr():
    import paper_2302_03245_amd as pr
    pr.lib()
    return pr


@pytest.mark.parametrize("residual,tol,slots,batch_min,groups", [("fp32", 1e-6, 16, 1, 0), ("fp64", 1e-9, 8, 1, 0),
                                                                 ("fp32", 1e-6, 16, 2, 0), ("fp64", 1e-9, 16, 3, 0),
                                                                 ("fp32", 1e-6, 16, 1, 4), ("fp64", 1e-9, 8, 2, 4)])
def test_mix_equals_alone(pr, residual, tol, slots, batch_min, groups):
    import torch
    graphs = [prgen.workload_rmat_small(seed=0), prgen.random_digraph(20011, 150000, seed=3, dangling_frac=0.2,
                                                                      unref_frac=0.1)]
    # groups: vertex groups for ordered sweeps (batched rounds turn ordered once they gather)
    dgs = [pr.upload(g.row_ptr, g.col, groups=groups) for g in graphs]
    srv = pr.Server(c=C, l1_tol=tol, residual=residual, slots=slots, sweeps_per_round=3, batch_min=batch_min)
    gids = [srv.add_graph(d) for d in dgs]
    rng = np.random.default_rng(5)
    queries = []
    for q in range(40):
        gi = int(rng.integers(0, 2))
        src = -1 if rng.random() < 0.35 else int(rng.integers(0, graphs[gi].n))
        queries.append((gi, src))
    outs, rids = [], []
    for q, (gi, src) in enumerate(queries):
        out = torch.empty(graphs[gi].n, dtype=torch.float64, device="cuda")
        outs.append(out)
        rids.append(srv.submit(gids[gi], src, out))
        if q % 7 == 6:
            time.sleep(0.003)  # later waves arrive while earlier queries are in flight
        if q >= 30:
            time.sleep(0.002)  # a trickle at the end: short queues, solved alone unless batch_min is 1
    stats = [srv.wait(r, timeout=120.0) for r in rids]
    s = srv.stats()
    print(f"server: {s}", flush=True)
    assert s["completed"] == len(queries)
    ref_cache = {}
    for q, ((gi, src), st) in enumerate(zip(queries, stats)):
        assert st["status"] == 0 and st["l1_bound"] <= tol
        got = outs[q].cpu().numpy()
        g = graphs[gi]
        key = (gi, src)
        if key not in ref_cache:
            p = None
            if src >= 0:
                p = np.zeros(g.n)
                p[src] = 1.0
            ref_cache[key] = oracle.power(g, C, p, tol=1e-13)[0]
        ref = ref_cache[key]
        assert l1(got, ref) <= tol, (q, gi, src, l1(got, ref))
        # the same query alone
        if src >= 0:
            alone = pr.ppr(dgs[gi], [src], c=C, l1_tol=tol, residual=residual)[0][0]
        else:
            alone = pr.ifp2(dgs[gi], c=C, l1_tol=tol, residual=residual)[0]
        assert l1(got, alone) <= 2 * tol
    srv.close()


def test_server_rejections(pr):
    import torch
    g = prgen.random_digraph(1000, 6000, seed=1, dangling_frac=0.2)
    dg = pr.upload(g.row_ptr, g.col)
    with pytest.raises(pr.PRError, match="slots"):
        pr.Server(slots=12)
    with pytest.raises(pr.PRError, match="batch_min"):
        pr.Server(batch_min=0)
    small = pr.Server(memory_budget=1024)
    with pytest.raises(pr.PRError, match="budget"):
        small.add_graph(dg)
    small.close()
    srv = pr.Server()
    gid = srv.add_graph(dg)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PRError, match="graph id"):
        srv.submit(gid + 5, 0, out)
    with pytest.raises(pr.PRError, match="source"):
        srv.submit(gid, g.n, out)
    rid = srv.submit(gid, 3, out)
    st = srv.wait(rid, timeout=60.0)
    assert st["status"] == 0
    with pytest.raises(pr.PRError, match="collected"):
        srv.wait(rid)
    srv.close()


def _reference(graphs, gi, src, cache):
    key = (gi, src)
    if key not in cache:
        g = graphs[gi]
        p = None
        if src >= 0:
            p = np.zeros(g.n)
            p[src] = 1.0
        cache[key] = oracle.power(g, C, p, tol=1e-13)[0]
    return cache[key]


def test_memory_admission(pr):
    """Queries are admitted by workspace footprint: under a budget with room for one
    single-query workspace the engines' batched runs narrow to single solves and the two
    engines take turns; with room for an 8-wide run a 16-query queue runs 8 wide.  Every
    result still matches the oracle, and device use never exceeds the budget."""
    import torch
    tol = 1e-6
    graphs = [prgen.workload_rmat_small(seed=0), prgen.random_digraph(20011, 150000, seed=3, dangling_frac=0.2,
                                                                      unref_frac=0.1)]
    dgs = [pr.upload(g.row_ptr, g.col) for g in graphs]
    # footprints, read from a server with room for everything (registration also builds
    # the batch plans and stop weights that stay on the graphs)
    big = pr.Server(c=C, l1_tol=tol, slots=16, batch_min=1)
    gids = [big.add_graph(d) for d in dgs]
    gb = big.stats()["graph_bytes"]
    one = [big.footprint(i, 1) for i in gids]
    w8 = [big.footprint(i, 8) for i in gids]
    w16 = [big.footprint(i, 16) for i in gids]
    with pytest.raises(pr.PRError, match="width"):
        big.footprint(gids[0], 4)
    big.close()
    print(f"graphs {gb} B, single {one}, 8-wide {w8}, 16-wide {w16}", flush=True)
    assert max(one) + 4096 < min(w8) and w8[1] + 4096 < w16[1]
    cache = {}
    rng = np.random.default_rng(11)

    def serve(budget, queries):
        srv = pr.Server(c=C, l1_tol=tol, slots=16, batch_min=1, sweeps_per_round=3, memory_budget=budget)
        ids = [srv.add_graph(d) for d in dgs]
        outs = [torch.empty(graphs[gi].n, dtype=torch.float64, device="cuda") for gi, _ in queries]
        rids = [srv.submit(ids[gi], src, out) for (gi, src), out in zip(queries, outs)]
        sts = [srv.wait(r, timeout=120.0) for r in rids]
        s = srv.stats()
        srv.close()
        print(f"budget {budget}: {s}", flush=True)
        assert s["completed"] == len(queries) and s["rejected"] == 0
        assert s["budget"] == budget and gb <= s["peak_bytes"] <= budget
        for (gi, src), st, out in zip(queries, sts, outs):
            assert st["status"] == 0 and st["l1_bound"] <= tol
            ref = _reference(graphs, gi, src, cache)
            assert l1(out.cpu().numpy(), ref) <= tol, (gi, src)
        return s

    # room for one single-query workspace: narrowed runs, engines waiting for each other
    qs = [(q % 2, -1 if q % 5 == 0 else int(rng.integers(0, graphs[q % 2].n))) for q in range(24)]
    s = serve(gb + max(one) + 4096, qs)
    assert s["narrowed_runs"] >= 1 and s["memory_waits"] >= 1
    # room for one 8-wide run on the second graph: a 16-query queue there runs 8 wide
    qs = [(1, int(rng.integers(0, graphs[1].n))) for _ in range(16)]
    s = serve(gb + w8[1] + 4096, qs)
    assert s["peak_bytes"] >= gb + w8[1]  # batched, 8 wide (16 wide would exceed the budget)


def test_memory_admission_rejects_graphs(pr):
    """A graph is registered only if it and one single-query workspace fit next to the
    graphs registered before it."""
    ga = prgen.random_digraph(3000, 20000, seed=4, dangling_frac=0.2)
    gb_ = prgen.random_digraph(5000, 40000, seed=5, dangling_frac=0.2)
    da, db = pr.upload(ga.row_ptr, ga.col), pr.upload(gb_.row_ptr, gb_.col)
    probe = pr.Server()
    ia = probe.add_graph(da)
    bytes_a = probe.stats()["graph_bytes"]
    one_a = probe.footprint(ia, 1)
    probe.close()
    srv = pr.Server(memory_budget=bytes_a + one_a + 1024)
    srv.add_graph(da)
    with pytest.raises(pr.PRError, match="budget"):
        srv.add_graph(db)
    s = srv.stats()
    assert s["graph_bytes"] == bytes_a and s["device_bytes"] <= s["budget"]
    srv.close()
