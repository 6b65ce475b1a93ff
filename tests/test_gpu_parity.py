"""GPU parity: the HIP path through the C ABI against the CPU oracle and the exact fixtures.

Tolerances: L1 <= 1e-9 with FP64 residuals, L1 <= 1e-6 with FP32 residuals, the
top-1000 ranking equal under the tie rule of conftest.topk_agree.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import prgen
from conftest import covered, l1, topk_agree

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
C = 0.85


@pytest.fixture(scope="module")
def pr():
    import paper_2302_03245_amd as pr
    pr.lib()
    return pr


def _say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------------------
# tiny graphs with known answers
# ----------------------------------------------------------------------------
def _closed_forms():
    out = []
    n = 37
    k = np.arange(1, n + 1)
    y = (1 - C ** k) / (1 - C)
    out.append(("chain37", prgen.from_edges(n, np.arange(n - 1), np.arange(1, n)), y / y.sum()))
    kk = 40
    e = np.full(kk + 1, 1 / (1 + kk + C * kk))
    e[0] = (1 + C * kk) / (1 + kk + C * kk)
    out.append(("in_star40", prgen.from_edges(kk + 1, np.arange(1, kk + 1), np.zeros(kk, int)), e))
    kk = 5000  # hub row longer than a merge-path tile
    e = np.full(kk + 1, (1 + C / kk) / (kk + 1 + C))
    e[0] = 1 / (kk + 1 + C)
    out.append(("out_star5000", prgen.from_edges(kk + 1, np.zeros(kk, int), np.arange(1, kk + 1)), e))
    e = np.full(kk + 1, 1 / (1 + kk + C * kk))
    e[0] = (1 + C * kk) / (1 + kk + C * kk)
    out.append(("in_star5000", prgen.from_edges(kk + 1, np.arange(1, kk + 1), np.zeros(kk, int)), e))
    out.append(("cycle100", prgen.from_edges(100, np.arange(100), (np.arange(100) + 1) % 100), np.full(100, 0.01)))
    out.append(("two", prgen.from_edges(2, [0], [1]), np.array([1, 1 + C]) / (2 + C)))
    out.append(("no_edges", prgen.from_edges(5, [], []), np.full(5, 0.2)))
    out.append(("single", prgen.from_edges(1, [], []), np.array([1.0])))
    out.append(("single_selfloop", prgen.from_edges(1, [0], [0]), np.array([1.0])))
    return out


CLOSED = _closed_forms()


@pytest.mark.parametrize("name,g,expect", CLOSED, ids=[c[0] for c in CLOSED])
@pytest.mark.parametrize("method", ["ifp1", "ifp2", "power"])
def test_closed_forms(pr, name, g, expect, method):
    _say(f"closed form {name} {method}")
    dg = pr.upload(g.row_ptr, g.col)
    for mode in ([None, "push", "pull", "list"] if method != "power" else [None]):
        if method == "power":
            # 1e-12: below that the order of the FP64 atomic adds into a hub row is visible in ||x' - x||
            pi, st = pr.power(dg, c=C, l1_tol=1e-12)
        else:
            pi, st = getattr(pr, method)(dg, c=C, xi=1e-15, mode=mode)
        assert st["status"] == 0
        assert l1(pi, expect) <= 1e-11, (mode, l1(pi, expect))
        assert abs(pi.sum() - 1) < 1e-13


GOLD = json.load(open(os.path.join(HERE, "golden", "exact_small.json")))["cases"]


@pytest.mark.parametrize("case", GOLD, ids=[c["name"] for c in GOLD])
def test_exact_fixtures(pr, case):
    _say(f"exact fixture {case['name']}")
    c = float(Fraction(case["c"]))
    p = None if case["p"] is None else np.array(case["p"], float)
    dg = pr.upload(np.array(case["row_ptr"], np.int64), np.array(case["col"], np.int32))
    ref = np.array(case["pi"])
    for fn in (pr.ifp1, pr.ifp2):
        for res, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
            # FP32 at xi = 1e-9 stops below FP32's rounding floor: the run verifies itself
            pi, st = fn(dg, p=p, c=c, xi=1e-15 if res == "fp64" else 1e-9, residual=res, verify=res == "fp32")
            covered(st, pi, ref, tol, ref_err=1e-15)
    pi, st = pr.power(dg, p=p, c=c, l1_tol=1e-12)
    assert l1(pi, ref) <= 1e-12


# ----------------------------------------------------------------------------
# random graphs spanning several tiles and a ragged tail
# ----------------------------------------------------------------------------
RANDOM = [
    ("rand_n3001", dict(n=3001, m=24000, seed=1, dangling_frac=0.2, unref_frac=0.1)),
    ("rand_n20011_selfloops_multi", dict(n=20011, m=150000, seed=2, self_loops=True, multi=True, dangling_frac=0.3)),
    ("rand_n70001", dict(n=70001, m=420000, seed=3, dangling_frac=0.15, unref_frac=0.1)),
]


@pytest.mark.parametrize("name,kw", RANDOM, ids=[r[0] for r in RANDOM])
def test_random_graphs(pr, name, kw):
    g = prgen.random_digraph(**kw)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col)
    info = dg.info()
    assert info["n"] == g.n and info["m"] == g.m
    for method in ("ifp1", "ifp2"):
        for mode in (None, "push", "pull", "list"):
            _say(f"{name} {method} mode={mode}")
            pi, st = getattr(pr, method)(dg, c=C, xi=1e-13, mode=mode)
            assert st["status"] == 0
            assert l1(pi, ref) <= 1e-9
            ok, swaps, eps = topk_agree(ref, pi, 1000, "fp64")
            assert ok, (swaps, eps)
            pi32, st32 = getattr(pr, method)(dg, c=C, l1_tol=1e-6, residual="fp32", mode=mode)
            assert st32["status"] == 0 and st32["l1_bound"] <= 1e-6
            covered(st32, pi32, ref, 1e-6)
    pi, st = pr.power(dg, c=C, l1_tol=1e-11)
    assert l1(pi, ref) <= 1e-9
    pi, st = pr.power(dg, c=C, l1_tol=1e-6, residual="fp32")
    covered(st, pi, ref, 1e-6)


@pytest.mark.parametrize("shift", [2, 3, 4])
def test_tile_sizes(pr, shift):
    """Every sweep tile size gives the same answer (hub rows spanning tiles included)."""
    g = prgen.workload_rmat_small(seed=4)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col, tile_shift=shift)
    for method in ("ifp1", "ifp2"):
        for mode in ("push", "pull"):
            pi, st = getattr(pr, method)(dg, c=C, xi=1e-13, mode=mode)
            assert l1(pi, ref) <= 1e-9
    pw, _ = pr.power(dg, c=C, l1_tol=1e-12)
    assert l1(pw, ref) <= 1e-11


def test_depth_epochs_on_a_dag(pr):
    """Gather sweeps on compacted in-edge lists (sources past their unreferenced depth
    dropped) give the oracle's answer; the epochs exist on a layered DAG."""
    g = prgen.workload_dag(n_layers=12, layer_size=3000, zmax=200, target_edges=300_000, back_frac=0.005, seed=2)
    dg = pr.upload(g.row_ptr, g.col)
    info = dg.info()
    assert info["epochs"] > 1 and info["max_depth"] >= 2
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    for method in ("ifp1", "ifp2"):
        for mode in (None, "pull"):
            pi, st = getattr(pr, method)(dg, c=C, xi=1e-13, mode=mode)
            assert st["status"] == 0
            assert l1(pi, ref) <= 1e-9
            pi32, st32 = getattr(pr, method)(dg, c=C, l1_tol=1e-6, residual="fp32", mode=mode)
            covered(st32, pi32, ref, 1e-6)
    p = prgen.random_p(g.n, seed=3, zero_frac=0.5)
    ref_p, _, _ = oracle.power(g, C, p, tol=1e-13)
    pi, _ = pr.ifp2(dg, p=p, c=C, xi=1e-13, mode="pull")
    assert l1(pi, ref_p) <= 1e-9


def test_rmat_small_workload(pr):
    """R-MAT n=10,000, 100,000 distinct edges, 10 % forced dangling, c=0.85, uniform p,
    xi=1e-12, FP64: IFP2 against the FP64 power method run to 1e-13."""
    _say("rmat small workload")
    g = prgen.workload_rmat_small(seed=0)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col)
    pi, st = pr.ifp2(dg, c=C, xi=1e-12)
    assert st["status"] == 0
    assert l1(pi, ref) <= 1e-9
    ok, swaps, eps = topk_agree(ref, pi, 1000, "fp64")
    assert ok, (swaps, eps)
    pi1, _ = pr.ifp1(dg, c=C, xi=1e-12)
    assert l1(pi1, ref) <= 1e-9
    assert topk_agree(ref, pi1, 1000, "fp64")[0]
    pw, _ = pr.power(dg, c=C, l1_tol=1e-12)
    assert l1(pw, ref) <= 1e-11
    # work: IFP2 pushes fewer edges than IFP1 at the same threshold
    _, st1 = pr.ifp1(dg, c=C, xi=1e-12, mode="push")
    _, st2 = pr.ifp2(dg, c=C, xi=1e-12, mode="push")
    assert st2["edges_processed"] < st1["edges_processed"]


def test_same_semantics_as_serial_when_nothing_moves(pr):
    """xi above every initial residual: no vertex pushes, IFP2's phase 2 alone decides
    the dangling values -- identical to the oracle with the same xi."""
    g = prgen.random_digraph(5000, 30000, seed=7, dangling_frac=0.3)
    dg = pr.upload(g.row_ptr, g.col)
    for method in ("ifp1", "ifp2"):
        pi, st = getattr(pr, method)(dg, c=C, xi=10.0)
        ref = getattr(oracle, method)(g, C, xi=10.0)["pi"]
        assert st["sweeps"] == 0
        np.testing.assert_allclose(pi, ref, rtol=1e-13, atol=0)


# ----------------------------------------------------------------------------
# personalisation, PPR, device buffers, literal IFP2, damping extremes
# ----------------------------------------------------------------------------
def test_personalized_p_host_and_device(pr):
    import torch
    g = prgen.workload_rmat_small(seed=1)
    p = prgen.random_p(g.n, seed=5, zero_frac=0.4)
    ref, _, _ = oracle.power(g, C, p, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col)
    pi, _ = pr.ifp2(dg, p=p * 7.0, c=C, xi=1e-12)  # p is normalised by its sum
    assert l1(pi, ref) <= 1e-9
    pt = torch.tensor(p, dtype=torch.float64, device="cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    pr.ifp1(dg, p=pt, c=C, xi=1e-12, out=out)
    torch.cuda.synchronize()
    assert l1(out.cpu().numpy(), ref) <= 1e-9
    pw, _ = pr.power(dg, p=pt, c=C, l1_tol=1e-12)
    assert l1(pw, ref) <= 1e-11


def test_upload_from_device_tensors(pr):
    import torch
    g = prgen.random_digraph(9000, 60000, seed=8, dangling_frac=0.2)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(torch.tensor(g.row_ptr, device="cuda"), torch.tensor(g.col, device="cuda"))
    pi, _ = pr.ifp2(dg, c=C, xi=1e-13)
    assert l1(pi, ref) <= 1e-9


def test_ppr_sources(pr):
    g = prgen.workload_rmat_small(seed=2)
    dg = pr.upload(g.row_ptr, g.col)
    deg = np.diff(g.row_ptr)
    srcs = [int(np.argmax(deg)), 17, int(np.where(deg == 0)[0][0])]  # hub, ordinary, dangling source
    out, stats = pr.ppr(dg, srcs, c=C, xi=1e-12)
    for r, s in enumerate(srcs):
        p = np.zeros(g.n)
        p[s] = 1.0
        ref, _, _ = oracle.power(g, C, p, tol=1e-13)
        _say(f"ppr source {s}: sweeps {stats[r]['sweeps']}")
        assert l1(out[r], ref) <= 1e-9
    out32, st32 = pr.ppr(dg, srcs[:1], c=C, l1_tol=1e-6, residual="fp32")
    p = np.zeros(g.n)
    p[srcs[0]] = 1.0
    covered(st32[0], out32[0], oracle.power(g, C, p, tol=1e-13)[0], 1e-6)


@pytest.mark.parametrize("mode", [None, "push", "pull", "list"])
def test_ppr_batches(pr, mode):
    """Twenty-one sources: one batch of sixteen column-interleaved vectors and one of
    five (width 8), each column against the oracle with p = e_s, FP64 and FP32 residuals."""
    g = prgen.workload_rmat_small(seed=5)
    dg = pr.upload(g.row_ptr, g.col)
    deg = np.diff(g.row_ptr)
    rng = np.random.default_rng(11)
    srcs = [int(np.argmax(deg)), int(np.where(deg == 0)[0][3])] + [int(x) for x in rng.choice(g.n, 19, replace=False)]
    out, stats = pr.ppr(dg, srcs, c=C, xi=1e-12, mode=mode)
    out32, stats32 = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32", mode=mode)
    for r, s in enumerate(srcs):
        p = np.zeros(g.n)
        p[s] = 1.0
        ref, _, _ = oracle.power(g, C, p, tol=1e-13)
        assert stats[r]["status"] == 0
        assert l1(out[r], ref) <= 1e-9, (r, s)
        assert stats32[r]["l1_bound"] <= 1e-6
        covered(stats32[r], out32[r], ref, 1e-6)


@pytest.mark.parametrize("gi", [0, 1])
def test_ppr_batch_ordered_sweeps(pr, gi):
    """Batches of sixteen and of five sources on graphs uploaded with four vertex groups
    turn to ordered sweeps once their columns' frontiers are dense; their S_N comes
    from the reserves' own sums.  Every column, FP64 to an empty frontier and FP32 to the
    certified L1 bound, against the oracle, and against the same batch kept synchronous
    (jacobi), which needs more sweeps.  Graph 1 has unreferenced vertices (gathers over
    later epochs' in-lists)."""
    g = [prgen.workload_rmat_small(seed=5),
         prgen.random_digraph(20011, 150000, seed=3, dangling_frac=0.2, unref_frac=0.1)][gi]
    dg = pr.upload(g.row_ptr, g.col, groups=4)
    assert dg.info()["groups"] == 4
    deg = np.diff(g.row_ptr)
    srcs = [int(x) for x in np.random.default_rng(21 + gi).choice(np.flatnonzero(deg > 0), 21, replace=False)]
    out, st = pr.ppr(dg, srcs, c=C, xi=1e-12)
    outj, stj = pr.ppr(dg, srcs, c=C, xi=1e-12, jacobi=True)
    out32, st32 = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32")
    out32j, st32j = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32", jacobi=True)
    sw = [sum(x["sweeps"] for x in z) for z in (st, stj, st32, st32j)]
    _say(f"ppr batch ordered / synchronous sweeps: FP64 {sw[0]} / {sw[1]}, FP32 {sw[2]} / {sw[3]}")
    assert sw[0] < sw[1] and sw[2] < sw[3]
    for r, s in enumerate(srcs):
        p = np.zeros(g.n)
        p[s] = 1.0
        ref, _, _ = oracle.power(g, C, p, tol=1e-13)
        assert st[r]["status"] == 0 and st32[r]["status"] == 0
        assert l1(out[r], ref) <= 1e-9 and l1(outj[r], ref) <= 1e-9, (r, s)
        assert st32[r]["l1_bound"] <= 1e-6
        covered(st32[r], out32[r], ref, 1e-6)
        covered(st32j[r], out32j[r], ref, 1e-6)


def _dyadic_graph(n, seed):
    """Random digraph whose out-degrees are powers of two (1, 2, 4, 8): with c = 1/2 every
    push weight c v / deg(i) is exact in FP64, so two sweeps that take the same vertices
    differ only in the order of their adds (rounding far below any threshold)."""
    rng = np.random.default_rng(seed)
    deg = np.where(rng.random(n) < 0.2, 0, 2 ** rng.integers(0, 4, n))
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, src.size)
    return prgen.from_edges(n, src, dst)


@pytest.mark.parametrize("method", ["ifp1", "ifp2"])
def test_list_sweeps_take_the_same_vertices(pr, method):
    """List sweeps (the frontier compacted into a list of ids between sweeps, scattered
    with returning atomics that append the targets crossing xi) take exactly the
    vertices the tile scatter takes, sweep by sweep (c = 1/2, power-of-two degrees, FP64:
    exact weights): same active vertices and edges in every sweep, and the same result up
    to the order of the adds."""
    g = _dyadic_graph(30011, seed=4)
    dg = pr.upload(g.row_ptr, g.col)
    fn = getattr(pr, method)
    pa, sa = fn(dg, c=0.5, xi=2.0 ** -20, mode="push", profile=True)
    ta = pr.last_trace()
    pb, sb = fn(dg, c=0.5, xi=2.0 ** -20, mode="list", profile=True)
    tb = pr.last_trace()
    _say(f"list vs tile scatter: sweeps {sa['sweeps']} / {sb['sweeps']}, pushes {sa['vertex_pushes']} / "
         f"{sb['vertex_pushes']}")
    assert sa["sweeps"] == sb["sweeps"]
    assert sa["vertex_pushes"] == sb["vertex_pushes"]
    assert sa["edges_processed"] == sb["edges_processed"]
    assert np.array_equal(ta["active"], tb["active"]) and np.array_equal(ta["edges"], tb["edges"])
    assert float(np.abs(pa - pb).max()) <= 1e-15
    ref = oracle.power(g, 0.5, tol=1e-13)[0]
    assert l1(pb, ref) <= 4 * sb["l1_bound"] + 1e-12
    dg.free()


def test_list_sweeps_sparse_then_dense(pr):
    """Single-source solves start with list sweeps and turn to dense sweeps as the
    frontier grows; a personalised p with a few non-zero entries drops into list sweeps
    once its synchronous sweeps thin out.  Results against the oracle, FP64 and FP32."""
    g = prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15, unref_frac=0.1)
    dg = pr.upload(g.row_ptr, g.col)
    deg = np.diff(g.row_ptr)
    srcs = [int(np.argmax(deg)), int(np.flatnonzero(deg == 1)[0]), 12345]
    for s in srcs:
        e = np.zeros(g.n)
        e[s] = 1.0
        ref = oracle.power(g, C, e, tol=1e-13)[0]
        out, sts = pr.ppr(dg, [s], c=C, xi=1e-13)
        assert sts[0]["status"] == 0 and l1(out[0], ref) <= 1e-9, s
        out32, sts32 = pr.ppr(dg, [s], c=C, l1_tol=1e-6, residual="fp32")
        covered(sts32[0], out32[0], ref, 1e-6)
    p = np.zeros(g.n)
    p[np.random.default_rng(1).choice(g.n, 5, replace=False)] = 1.0
    ref = oracle.power(g, C, p, tol=1e-13)[0]
    for method in ("ifp1", "ifp2"):
        pi, st = getattr(pr, method)(dg, p=p, c=C, xi=1e-13)
        assert st["status"] == 0 and l1(pi, ref) <= 1e-9, method
    dg.free()


def _row_weights(g, c, iters=16):
    """f_j: L1 mass a unit at j adds to (I - cP)^{-1} (dangling vertices absorbing),
    as the library bounds it: 1 at a dangling j; 1 + c delta_j + (c / deg j) sum of f
    over j's non-dangling out-neighbours, iterated `iters` times from 1 / (1 - c)."""
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = np.asarray(g.col, dtype=np.int64)
    nd = deg > 0
    keep = nd[dst]
    dsafe = np.maximum(deg, 1)
    delta = np.where(nd, 1.0 - np.bincount(src[keep], minlength=g.n) / dsafe, 0.0)
    f = np.where(nd, 1.0 / (1.0 - c), 1.0)
    for _ in range(iters + 1):
        acc = np.bincount(src[keep], weights=f[dst[keep]], minlength=g.n)
        f = np.where(nd, 1.0 + c * delta + c * acc / dsafe, 1.0)
    return f


def _verified_numpy(g, pi, c, p, f):
    """The smallest of the check's bounds (without its rounding terms): ||r||_1 / (1 - c)
    with r = P'' pi - pi, and 2 sum_j f_j |beta p_j - ((I - cP) pi)_j| / sum(pi) at beta =
    c d^T pi + (1 - c) sum(pi) and at beta = the ratio pi_j / p_j summed over the vertices
    without in-edges; each + |sum(pi) - 1|."""
    import scipy.sparse as sp
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    inv = np.zeros(g.n)
    inv[deg > 0] = 1.0 / deg[deg > 0]
    P = sp.csr_matrix((inv[src], (g.col, src)), shape=(g.n, g.n))
    cp = c * (P @ pi)
    b = c * pi[deg == 0].sum() + (1 - c) * pi.sum()
    r = np.abs(cp + b * p - pi)
    best = min(r.sum() / (1 - c), 2 * float((f * r).sum()) / pi.sum())
    noin = np.bincount(np.asarray(g.col, dtype=np.int64), minlength=g.n) == 0
    if p[noin].sum() > 0:
        beta = pi[noin].sum() / p[noin].sum()
        best = min(best, 2 * float((f * np.abs(cp + beta * p - pi)).sum()) / pi.sum())
    return best + abs(pi.sum() - 1)


@pytest.mark.parametrize("residual", ["fp64", "fp32"])
def test_verified_bound(pr, residual):
    """PR_VERIFY: the a-posteriori bound -- the smaller of ||P'' pi - pi||_1 / (1 - c) and
    the row-weighted 2 sum_j f_j |r_j| / sum(pi), each + |sum(pi) - 1| (plus the rounding
    of the check) -- is computed as defined (against the same quantities in numpy from
    the returned vector) and bounds the distance to the oracle, for IFP1, IFP2 (folded
    and literal), the power method and single-source PPR."""
    g = prgen.random_digraph(20011, 150000, seed=2, self_loops=True, multi=True, dangling_frac=0.3)
    ref, _, delta = oracle.power(g, C, tol=1e-13)
    ref_err = C / (1 - C) * delta
    dg = pr.upload(g.row_ptr, g.col)
    u = np.full(g.n, 1.0 / g.n)
    f = _row_weights(g, C)
    tol = 1e-6 if residual == "fp32" else 1e-10
    runs = [("ifp1", lambda: pr.ifp1(dg, c=C, l1_tol=tol, residual=residual, verify=True)),
            ("ifp2", lambda: pr.ifp2(dg, c=C, l1_tol=tol, residual=residual, verify=True)),
            ("ifp2_literal", lambda: pr.ifp2(dg, c=C, l1_tol=tol, residual=residual, literal=True, verify=True)),
            ("power", lambda: pr.power(dg, c=C, l1_tol=tol, residual=residual, verify=True))]
    for name, run in runs:
        pi, st = run()
        d = l1(pi, ref)
        own = _verified_numpy(g, pi, C, u, f)
        _say(f"{name} {residual}: L1 {d:.3e} bound {st['l1_bound']:.3e} verified {st['l1_verified']:.3e} "
             f"(numpy {own:.3e}) launches {st['launches']}")
        assert st["status"] == 0
        assert st["l1_verified"] >= d - ref_err, (name, st["l1_verified"], d)
        assert st["l1_verified"] <= tol
        # the library adds the rounding of its own check (about (in-degree + reduction
        # depth) x 2^-53 of the mass per row, / (1 - c)) and stores its weights rounded
        # up in FP32; numpy's figure has neither
        assert own * (1 - 1e-9) <= st["l1_verified"] <= own * (1 + 1e-3) + 1e-12, (name, st["l1_verified"], own)
        assert st["launches"] > 0
    s = int(np.argmax(np.diff(g.row_ptr)))
    e = np.zeros(g.n)
    e[s] = 1.0
    ref_s, _, delta_s = oracle.power(g, C, e, tol=1e-13)
    out, sts = pr.ppr(dg, [s], c=C, l1_tol=tol, residual=residual, verify=True)
    own = _verified_numpy(g, out[0], C, e, f)
    assert sts[0]["l1_verified"] >= l1(out[0], ref_s) - C / (1 - C) * delta_s
    assert own * (1 - 1e-9) <= sts[0]["l1_verified"] <= own * (1 + 1e-3) + 1e-12
    dg.free()


def test_ppr_failing_later_batch_writes_nothing(pr):
    """A pr_ppr call whose second batch fails (testing hook: as if that batch's workspace
    could not be allocated) returns the negative status and leaves every output row and
    stats entry untouched, for host and device outputs; the same call without the hook
    then writes every row, each equal to the oracle's."""
    import torch
    g = prgen.workload_rmat_small(seed=5)
    dg = pr.upload(g.row_ptr, g.col)
    rng = np.random.default_rng(3)
    srcs = [int(x) for x in rng.choice(g.n, 20, replace=False)]  # a batch of 16, then one of 4
    sentinel = -7.25
    host = np.full((len(srcs), g.n), sentinel)
    dev = torch.full((len(srcs), g.n), sentinel, dtype=torch.float64, device="cuda")
    for out in (host, dev):
        pr.debug_fail_ppr_batch(1)
        with pytest.raises(pr.PRError) as ei:
            pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32", out=out)
        assert ei.value.status == pr.PR_ENOMEM
        vals = out.cpu().numpy() if hasattr(out, "cpu") else out
        assert np.all(vals == sentinel)
    # the hook is cleared by the failing call: the next call succeeds
    out, sts = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32", out=dev)
    got = dev.cpu().numpy()
    refs = []
    for s in srcs:
        p = np.zeros(g.n)
        p[s] = 1.0
        refs.append((g, C, p, 1e-13))
    from conftest import oracle_many
    for r, ref in enumerate(oracle_many(refs)):
        assert sts[r]["status"] == 0
        assert l1(got[r], ref) <= 1e-6, r
    dg.free()


def test_tune_busy_while_served(pr):
    """pr_graph_tune rebuilds the graph's plans, so it refuses (PR_EBUSY) while a query
    server holds the graph, and works again once the server is gone."""
    g = prgen.workload_rmat_small(seed=6)
    dg = pr.upload(g.row_ptr, g.col)
    srv = pr.Server(c=C, l1_tol=1e-6, residual="fp32", slots=8)
    try:
        srv.add_graph(dg)
        with pytest.raises(pr.PRError) as ei:
            pr.tune(dg, c=C, l1_tol=1e-6, residual="fp32", reps=1)
        assert ei.value.status == pr.PR_EBUSY
    finally:
        srv.close()
    rep = pr.tune(dg, c=C, l1_tol=1e-6, residual="fp32", reps=1)
    assert rep["candidates"]
    pi, st = pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32")
    assert st["status"] == 0
    dg.free()


def _edge_free_run(n_leaves=20000):
    """Vertex 0 -> 1 and every leaf v >= 1 -> 0: all vertices have out-edges, and rows
    2 .. n_leaves have no in-edge, so most gather tiles hold only row ends (a tile of
    IPB items then spans IPB + 1 rows, of which the last has no item in it)."""
    src = np.concatenate([[0], np.arange(1, n_leaves + 1)])
    dst = np.concatenate([[1], np.zeros(n_leaves, int)])
    return prgen.from_edges(n_leaves + 1, src, dst)


@pytest.mark.parametrize("shift", [2, 3, 4])
def test_tiles_of_row_ends_only(pr, shift):
    g = _edge_free_run()
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col, tile_shift=shift)
    for method in ("ifp1", "ifp2"):
        pi, st = getattr(pr, method)(dg, c=C, xi=1e-13, mode="pull")
        _say(f"shift {shift} {method}: sweeps {st['sweeps']} L1 {l1(pi, ref):.2e}")
        assert st["status"] == 0 and l1(pi, ref) <= 1e-9
        pi32, st32 = getattr(pr, method)(dg, c=C, l1_tol=1e-6, residual="fp32", mode="pull")
        assert st32["l1_bound"] <= 1e-6
        covered(st32, pi32, ref, 1e-6)
    pw, _ = pr.power(dg, c=C, l1_tol=1e-12)
    assert l1(pw, ref) <= 1e-11
    dg.free()


def test_batched_tiles_of_row_ends_only(pr):
    """The batched gather (128- and 256-item tiles for 16 and 8 columns) over the same
    runs of rows without in-edges: every column against the oracle's PPR."""
    g = _edge_free_run()
    dg = pr.upload(g.row_ptr, g.col)
    for srcs in ([0, 1, 2, 7, 19999, 20000] + list(range(100, 110)), [0, 5, 20000]):
        out, stats = pr.ppr(dg, srcs, c=C, xi=1e-12, mode="pull")
        out32, stats32 = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32", mode="pull")
        for r, s in enumerate(srcs):
            p = np.zeros(g.n)
            p[s] = 1.0
            ref, _, _ = oracle.power(g, C, p, tol=1e-13)
            assert stats[r]["status"] == 0 and l1(out[r], ref) <= 1e-9, (len(srcs), s)
            assert stats32[r]["l1_bound"] <= 1e-6, (len(srcs), s)
            covered(stats32[r], out32[r], ref, 1e-6)
    dg.free()


def test_literal_ifp2_matches_oracle_literal(pr):
    g = prgen.random_digraph(4000, 30000, seed=9, dangling_frac=0.25)
    dg = pr.upload(g.row_ptr, g.col)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    pi, st = pr.ifp2(dg, c=C, xi=1e-13, literal=True)
    assert l1(pi, ref) <= 1e-9
    assert st["l1_bound"] >= l1(pi, ref)


@pytest.mark.parametrize("c", [0.01, 0.5, 0.99])
def test_damping_extremes(pr, c):
    g = prgen.random_digraph(3000, 20000, seed=10, dangling_frac=0.2)
    ref, _, _ = oracle.power(g, c, tol=1e-14)
    dg = pr.upload(g.row_ptr, g.col)
    pi, st = pr.ifp2(dg, c=c, l1_tol=1e-10)
    assert st["status"] == 0
    assert l1(pi, ref) <= max(st["l1_bound"], 1e-12)
    pw, _ = pr.power(dg, c=c, l1_tol=1e-10)
    assert l1(pw, ref) <= 1e-10


def test_duplicates_counted_and_dedupe(pr):
    g = prgen.random_digraph(2000, 16000, seed=11, multi=True, self_loops=True, dangling_frac=0.1)
    assert np.any(np.diff(g.col) == 0)
    dg = pr.upload(g.row_ptr, g.col)
    pi, _ = pr.ifp2(dg, c=C, xi=1e-13)
    assert l1(pi, oracle.power(g, C, tol=1e-13)[0]) <= 1e-9
    dd = pr.upload(g.row_ptr, g.col, dedupe=True)
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    key = np.unique(src.astype(np.int64) * g.n + g.col)
    gu = prgen.from_edges(g.n, key // g.n, key % g.n)
    assert dd.m == gu.m
    pi, _ = pr.ifp2(dd, c=C, xi=1e-13)
    assert l1(pi, oracle.power(gu, C, tol=1e-13)[0]) <= 1e-9


def test_max_sweeps_gives_bounded_estimate(pr):
    g = prgen.workload_rmat_small(seed=3)
    ref, _, _ = oracle.power(g, C, tol=1e-13)
    dg = pr.upload(g.row_ptr, g.col)
    pi, st = pr.ifp2(dg, c=C, xi=1e-12, max_sweeps=3)
    assert st["status"] == 1 and st["sweeps"] == 3
    assert abs(pi.sum() - 1) < 1e-12
    assert l1(pi, ref) <= st["l1_bound"]
    pw, stp = pr.power(dg, c=C, l1_tol=1e-14, max_sweeps=2)
    assert stp["status"] == 1
    assert l1(pw, ref) <= stp["l1_bound"] + 1e-15


def test_invalid_arguments_on_gpu(pr):
    g = prgen.random_digraph(100, 500, seed=12)
    bad = g.col.copy()
    bad[3] = 100
    with pytest.raises(pr.PRError, match="out of"):
        pr.upload(g.row_ptr, bad)
    dg = pr.upload(g.row_ptr, g.col)
    with pytest.raises(pr.PRError, match="c must"):
        pr.ifp2(dg, c=1.0)
    with pytest.raises(pr.PRError, match="xi must"):
        pr.ifp2(dg, xi=0.0)
    with pytest.raises(pr.PRError, match="l1_tol"):
        pr.ifp2(dg, l1_tol=-1.0)
    p = np.ones(100)
    p[5] = -1
    with pytest.raises(pr.PRError, match="negative"):
        pr.ifp2(dg, p=p)
    with pytest.raises(pr.PRError, match="sum"):
        pr.ifp2(dg, p=np.zeros(100))
    with pytest.raises(pr.PRError, match="source"):
        pr.ppr(dg, [100])
    # outputs stay untouched on a negative status
    import torch
    out = torch.full((100,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PRError, match="negative"):
        pr.ifp2(dg, p=p, out=out)
    with pytest.raises(pr.PRError, match="c must"):
        pr.power(dg, c=0.0, out=out)
    assert bool((out == 7.0).all())
    host = np.full(100, 7.0)
    with pytest.raises(pr.PRError, match="l1_tol"):
        pr.ifp1(dg, l1_tol=-1.0, out=host)
    assert (host == 7.0).all()
    # the graph still works after the rejected calls
    pi, _ = pr.ifp2(dg, c=C, xi=1e-13)
    assert l1(pi, oracle.power(g, C, tol=1e-13)[0]) <= 1e-9


def test_equation_residual_and_bounds(pr):
    """A-posteriori check without the oracle: ||pi - c P pi - gamma p||_1 with
    gamma = 1 - c + c d^T pi (section 3.1), sum 1, pi >= (1-c) p."""
    import scipy.sparse as sp
    g = prgen.random_digraph(50000, 400000, seed=13, dangling_frac=0.2, unref_frac=0.1)
    dg = pr.upload(g.row_ptr, g.col)
    pi, st = pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32")
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    P = sp.csr_matrix((1.0 / deg[src], (g.col, src)), shape=(g.n, g.n))
    gamma = 1 - C + C * pi[deg == 0].sum()
    res = np.abs(pi - C * (P @ pi) - gamma / g.n).sum()
    assert res <= 2 * st["l1_bound"]
    assert abs(pi.sum() - 1) < 1e-12
    assert np.all(pi >= (1 - C) / g.n * (1 - 1e-6))


@pytest.mark.parametrize("groups", [2, 4, 15])
def test_group_gathers_over_reached_rows(pr, groups):
    """Ordered sweeps whose group gathers walk only the rows each group reaches (the
    default) and every row (PR_GROUP_ALL_ROWS) take the same vertices: same sweeps and
    pushes, results equal up to rounding order, both at the oracle; the autotuner times
    both forms when ordered sweeps win."""
    for g in (prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15, unref_frac=0.1),
              prgen.workload_dag(n_layers=12, layer_size=3000, zmax=200, target_edges=300_000, back_frac=0.005,
                                 seed=2)):
        ref, _, _ = oracle.power(g, C, tol=1e-13)
        dr = pr.upload(g.row_ptr, g.col, groups=groups)
        da = pr.upload(g.row_ptr, g.col, groups=groups, group_rows=False)
        for method in (pr.ifp2, pr.ifp1):
            pr_, sr = method(dr, c=C, xi=1e-13)
            pa, sa = method(da, c=C, xi=1e-13)
            _say(f"group rows {groups} {method.__name__} n {g.n}: sweeps {sr['sweeps']} / {sa['sweeps']}")
            assert sr["status"] == 0 and sa["status"] == 0
            assert sr["sweeps"] == sa["sweeps"] and sr["vertex_pushes"] == sa["vertex_pushes"]
            assert l1(pr_, pa) <= 1e-13 and l1(pr_, ref) <= 1e-9
            for residual, tol in (("fp32", 1e-6), ("fp64", 1e-10)):
                po, so = method(dr, c=C, l1_tol=tol, residual=residual)
                assert so["status"] == 0 and so["l1_bound"] <= tol and l1(po, ref) <= tol
        rep = pr.tune(da, c=C, l1_tol=1e-6, residual="fp32", reps=1)
        forms = {(cand["ordered"], cand["group_rows"]) for cand in rep["candidates"]}
        if rep["chosen"]["ordered"]:
            assert {(True, True), (True, False)} <= forms, rep
        pt, stt = pr.ifp2(da, c=C, l1_tol=1e-6, residual="fp32")
        assert stt["status"] == 0
        covered(stt, pt, ref, 1e-6)
        dr.free()
        da.free()


@pytest.mark.parametrize("groups", [1, 2, 4, 8, 15])
def test_ordered_sweeps(pr, groups):
    """Global IFP2 with ordered sweeps (the vertex groups take their residuals one after
    another within a sweep) reaches the oracle's answer with the same certificate as
    synchronous sweeps, and in no more sweeps."""
    for g in (prgen.workload_rmat_small(seed=0), prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15,
                                                                        unref_frac=0.1),
              prgen.workload_dag(n_layers=12, layer_size=3000, zmax=200, target_edges=300_000, back_frac=0.005,
                                 seed=2)):
        _say(f"ordered sweeps: groups {groups}, n {g.n}")
        ref, _, _ = oracle.power(g, C, tol=1e-13)
        dg = pr.upload(g.row_ptr, g.col, groups=groups)
        pi, st = pr.ifp2(dg, c=C, xi=1e-13)
        assert st["status"] == 0
        assert l1(pi, ref) <= 1e-9
        ok, swaps, eps = topk_agree(ref, pi, 1000, "fp64")
        assert ok, (swaps, eps)
        for residual, tol in (("fp32", 1e-6), ("fp64", 1e-10)):
            po, so = pr.ifp2(dg, c=C, l1_tol=tol, residual=residual)
            pj, sj = pr.ifp2(dg, c=C, l1_tol=tol, residual=residual, jacobi=True)
            assert so["status"] == 0 and so["l1_bound"] <= tol and sj["l1_bound"] <= tol
            covered(so, po, ref, tol)
            covered(sj, pj, ref, tol)
            assert l1(po, pj) <= 2 * tol
            assert abs(po.sum() - 1) < 1e-12
            if groups == 1:
                assert so["sweeps"] == sj["sweeps"]
            else:
                assert so["sweeps"] <= sj["sweeps"], (so["sweeps"], sj["sweeps"])
        pl, sl = pr.ifp2(dg, c=C, xi=1e-13, literal=True)
        assert l1(pl, ref) <= 1e-9 and sl["l1_bound"] >= l1(pl, ref)
        # IFP1 orders its sweeps the same way, gathering into every vertex
        p1, s1 = pr.ifp1(dg, c=C, xi=1e-13)
        assert s1["status"] == 0 and l1(p1, ref) <= 1e-9
        for residual, tol in (("fp32", 1e-6), ("fp64", 1e-10)):
            po, so = pr.ifp1(dg, c=C, l1_tol=tol, residual=residual)
            pj, sj = pr.ifp1(dg, c=C, l1_tol=tol, residual=residual, jacobi=True)
            assert so["status"] == 0 and so["l1_bound"] <= tol and sj["l1_bound"] <= tol
            covered(so, po, ref, tol)
            covered(sj, pj, ref, tol)
            if groups == 1:
                assert so["sweeps"] == sj["sweeps"]
            else:
                assert so["sweeps"] <= sj["sweeps"], (so["sweeps"], sj["sweeps"])


def test_autotune_keeps_results(pr):
    """The autotuner times every tile size with synchronous and ordered sweeps, keeps the
    fastest, and every solve afterwards still gives the oracle's answer."""
    for g, groups in ((prgen.workload_rmat_small(seed=0), 4),
                      (prgen.workload_dag(n_layers=12, layer_size=3000, zmax=200, target_edges=300_000,
                                          back_frac=0.005, seed=2), 4),
                      (prgen.random_digraph(20011, 150000, seed=2, dangling_frac=0.3), 0)):
        ref, _, _ = oracle.power(g, C, tol=1e-13)
        dg = pr.upload(g.row_ptr, g.col, groups=groups)
        rep = pr.tune(dg, c=C, l1_tol=1e-6, residual="fp32", reps=1)
        _say(f"tune n={g.n}: {rep}")
        cands = rep["candidates"]
        # small graphs get no groups by default; with groups, the other form of the group
        # gathers and then 3, 6 and 8 groups in both forms are timed at the tile size of the
        # fastest ordered candidate among the first six
        if groups == 0:
            assert len(cands) == 3
        else:
            first = min((x for x in cands[:6] if x["ordered"]), key=lambda x: x["ms"])
            extra = cands[6:]
            assert 1 <= len(extra) <= 7, rep
            assert all(x["tile_shift"] == first["tile_shift"] and x["ordered"] for x in extra), rep
            assert {x["groups"] for x in extra} <= {3, 4, 6, 8}, rep
            assert {(x["groups"], x["group_rows"]) for x in cands if x["ordered"]} >= {(4, True), (4, False)}
        assert all(x["groups"] == 1 for x in cands if not x["ordered"])
        assert sorted({x["tile_shift"] for x in cands}) == [2, 3, 4]
        assert rep["chosen"]["ms"] == min(x["ms"] for x in cands)
        info = dg.info()
        assert info["tile_items"] == 256 << rep["chosen"]["tile_shift"]
        assert info["ordered"] == int(rep["chosen"]["ordered"])
        if rep["chosen"]["ordered"]:
            assert info["groups"] == rep["chosen"]["groups"]
            # batched solves: a 16-source PPR batch timed both ways, the faster kept
            bm = rep["batch_ms"]
            assert rep["batch_ordered"] in (0, 1) and bm["ordered"] > 0 and bm["synchronous"] > 0, rep
            assert (bm["ordered"] <= bm["synchronous"]) == (rep["batch_ordered"] == 1), rep
        else:
            assert rep["batch_ordered"] == -1, rep
        for method in ("ifp1", "ifp2"):
            for mode in (None, "push", "pull", "list"):
                pi, st = getattr(pr, method)(dg, c=C, xi=1e-13, mode=mode)
                assert l1(pi, ref) <= 1e-9, (method, mode)
        pi, st = pr.ifp2(dg, c=C, l1_tol=1e-6, residual="fp32")
        assert st["l1_bound"] <= 1e-6
        covered(st, pi, ref, 1e-6)
        pw, _ = pr.power(dg, c=C, l1_tol=1e-11)
        assert l1(pw, ref) <= 1e-9
        srcs = [0, g.n // 2, g.n - 1]
        out, sts = pr.ppr(dg, srcs, c=C, xi=1e-13)
        for r, s in enumerate(srcs):
            p = np.zeros(g.n)
            p[s] = 1.0
            assert l1(out[r], oracle.power(g, C, p, tol=1e-13)[0]) <= 1e-9
        # a batch of sixteen under the batched sweeps the tuner kept (the gate only: a batched
        # FP32 column does not verify itself, and one whose residuals all drain to zero
        # reports an estimate of 0 against an error of FP32 rounding, about 1e-9)
        deg = np.diff(g.row_ptr)
        srcs = [int(x) for x in np.random.default_rng(3).choice(np.flatnonzero(deg > 0), 16, replace=False)]
        out, sts = pr.ppr(dg, srcs, c=C, l1_tol=1e-6, residual="fp32")
        for r, s in enumerate(srcs[:4]):
            p = np.zeros(g.n)
            p[s] = 1.0
            assert sts[r]["status"] == 0 and sts[r]["l1_bound"] <= 1e-6
            assert l1(out[r], oracle.power(g, C, p, tol=1e-13)[0]) <= 1e-6
    o = pr._opts(C, 1e-12, 1e-6, "fp32", 0, None, False, "push", False)
    assert pr.lib().pr_graph_tune(dg.handle, o, 1, None) == pr.PR_EINVAL
    assert "automatic" in pr.lib().pr_last_error().decode()


def test_ordered_sweeps_after_a_sparse_start(pr):
    """Single-source PPR and personalised p on a graph with vertex groups: the solve starts
    with synchronous sweeps and turns to ordered sweeps once a sweep gathers; the result
    matches the oracle and takes no more sweeps than synchronous sweeps alone."""
    g = prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15, unref_frac=0.1)
    dg = pr.upload(g.row_ptr, g.col, groups=4)
    deg = np.diff(g.row_ptr)
    for s in np.flatnonzero(deg > 0)[[0, 500, 20000]]:
        p = np.zeros(g.n)
        p[s] = 1.0
        ref = oracle.power(g, C, p, tol=1e-13)[0]
        out, st = pr.ppr(dg, [int(s)], c=C, xi=1e-13)
        outj, stj = pr.ppr(dg, [int(s)], c=C, xi=1e-13, jacobi=True)
        assert l1(out[0], ref) <= 1e-9 and l1(outj[0], ref) <= 1e-9
        assert st[0]["sweeps"] <= stj[0]["sweeps"] + 1, (st[0]["sweeps"], stj[0]["sweeps"])
        o32, s32 = pr.ppr(dg, [int(s)], c=C, l1_tol=1e-6, residual="fp32")
        assert s32[0]["l1_bound"] <= 1e-6
        covered(s32[0], o32[0], ref, 1e-6)
    p = prgen.random_p(g.n, seed=4, zero_frac=0.3)
    ref = oracle.power(g, C, p, tol=1e-13)[0]
    for method in (pr.ifp2, pr.ifp1):
        pi, st = method(dg, p=p, c=C, l1_tol=1e-10)
        pj, sj = method(dg, p=p, c=C, l1_tol=1e-10, jacobi=True)
        assert st["l1_bound"] <= 1e-10 and l1(pi, ref) <= 1e-10 and l1(pj, ref) <= 1e-10
        assert st["sweeps"] < sj["sweeps"], (method.__name__, st["sweeps"], sj["sweeps"])
    # IFP1 from a single source: the frontier starts with one vertex
    e = np.zeros(g.n)
    e[int(np.flatnonzero(deg > 0)[7])] = 1.0
    ref = oracle.power(g, C, e, tol=1e-13)[0]
    pi, st = pr.ifp1(dg, p=e, c=C, xi=1e-13)
    assert st["status"] == 0 and l1(pi, ref) <= 1e-9


def test_concurrent_solves_on_one_graph(pr):
    """The graph is read-only after upload: solves from several host threads, each on its
    own stream, share one handle (the second takes a workspace of its own) and give the
    answers of the same solves run one after another."""
    import threading

    import torch
    g = prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15, unref_frac=0.1)
    dg = pr.upload(g.row_ptr, g.col, groups=4)
    deg = np.diff(g.row_ptr)
    srcs = [int(x) for x in np.flatnonzero(deg > 0)[[3, 300, 3000]]]
    ref_glob, _ = pr.ifp2(dg, c=C, l1_tol=1e-9)
    ref_ppr, _ = pr.ppr(dg, srcs, c=C, l1_tol=1e-9)
    ref_pow, _ = pr.power(dg, c=C, l1_tol=1e-9)
    results, errors = {}, []

    def work(name, fn):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    results[name] = fn(s)
        except Exception as e:  # reported below, on the main thread
            errors.append((name, repr(e)))

    jobs = {
        "ifp2": lambda s: pr.ifp2(dg, c=C, l1_tol=1e-9, stream=s.cuda_stream)[0],
        "ppr": lambda s: pr.ppr(dg, srcs, c=C, l1_tol=1e-9, stream=s.cuda_stream)[0],
        "power": lambda s: pr.power(dg, c=C, l1_tol=1e-9, stream=s.cuda_stream)[0],
        "ifp2_b": lambda s: pr.ifp2(dg, c=C, l1_tol=1e-9, stream=s.cuda_stream)[0],
    }
    threads = [threading.Thread(target=work, args=(k, f)) for k, f in jobs.items()]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not errors, errors
    assert l1(results["ifp2"], ref_glob) <= 1e-12 and l1(results["ifp2_b"], ref_glob) <= 1e-12
    assert l1(results["power"], ref_pow) <= 1e-12
    for r in range(len(srcs)):
        assert l1(results["ppr"][r], ref_ppr[r]) <= 1e-12
