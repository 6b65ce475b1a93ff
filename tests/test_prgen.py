"""Input generators: determinism and the structural properties of each recipe (no GPU)."""
import os
import subprocess
import sys

import numpy as np

import prgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_csr(g, allow_self=False):
    assert g.row_ptr[0] == 0 and np.all(np.diff(g.row_ptr) >= 0)
    assert g.col.dtype == np.int32 and g.row_ptr.dtype == np.int64
    assert np.all((g.col >= 0) & (g.col < g.n))
    deg = np.diff(g.row_ptr)
    src = np.repeat(np.arange(g.n), deg)
    key = src * g.n + g.col
    assert np.all(np.diff(key) > 0), "rows sorted, no repeated edge"
    if not allow_self:
        assert not np.any(src == g.col)


def test_rmat_small_recipe():
    g = prgen.workload_rmat_small()
    _check_csr(g)
    s = prgen.stats(g)
    assert s["n"] == 10_000
    # 100,000 distinct edges before the dangling drop; 10 % of vertices forced dangling
    assert 80_000 < s["m"] < 100_000
    assert s["n_d"] >= 1_000
    g2 = prgen.workload_rmat_small()
    assert np.array_equal(g.row_ptr, g2.row_ptr) and np.array_equal(g.col, g2.col)
    g3 = prgen.workload_rmat_small(seed=1)
    assert not np.array_equal(g.col[:1000], g3.col[:1000])


def test_rmat_recipe_small_scale():
    g = prgen.workload_rmat(scale=12, edge_factor=16)
    _check_csr(g)
    s = prgen.stats(g)
    assert s["n_d"] >= int(0.15 * g.n)
    assert s["n_u"] >= int(0.10 * g.n)


def test_rmat_thread_count_independent():
    code = ("import sys; sys.path.insert(0, %r); import prgen, hashlib; g = prgen.workload_rmat(scale=13);"
            "print(hashlib.sha1(g.row_ptr.tobytes() + g.col.tobytes()).hexdigest())" % ROOT)
    outs = []
    for threads in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        env.pop("PRGEN_CACHE", None)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   text=True, check=True).stdout.strip())
    assert outs[0] == outs[1]


def test_dag_recipe_small():
    L, w = 8, 500
    g = prgen.workload_dag(n_layers=L, layer_size=w, zmax=100, target_edges=20_000, back_frac=0.02)
    _check_csr(g)
    s = prgen.stats(g)
    deg = np.diff(g.row_ptr)
    # only the last layer is dangling; the first layer is unreferenced
    assert s["n_d"] == w
    assert s["n_u"] >= w
    assert abs((s["m"] - round(0.02 * 20_000)) - 20_000) <= 0.002 * 20_000 + 5
    assert deg.max() <= 100 + 50


def _mix64(z):
    M = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def _rmat_exact_reference(n, scale, target_m, n_dangling, seed, wl, a=0.57, b=0.19, c=0.19):
    """The definition of the exact-count R-MAT recipe, written sequentially: draws in
    counter order, rejected when an endpoint is >= n, a self-loop or a repeat, until
    target_m distinct edges; then the dangling drop and the relabel permutation."""
    M = (1 << 64) - 1
    G = 0x9E3779B97F4A7C15
    key = lambda purpose: _mix64((seed * G & M) ^ _mix64((wl << 32) | purpose))
    at = lambda k, ctr: _mix64((k + (ctr + 1) * G) & M)
    ke, kd, kr = key(0), key(1), key(3)

    def perm(size, k):
        p = list(range(size))
        for i in range(size - 1, 0, -1):
            j = (at(k, i) * (i + 1)) >> 64
            p[i], p[j] = p[j], p[i]
        return p
    seen, edges, ctr = set(), [], 0
    while len(edges) < target_m:
        s = t = 0
        for lvl in range(scale):
            u = (at(ke, ctr * 64 + lvl) >> 11) * 2.0 ** -53
            bs, bt = (0, 0) if u < a else (0, 1) if u < a + b else (1, 0) if u < a + b + c else (1, 1)
            s, t = (s << 1) | bs, (t << 1) | bt
        ctr += 1
        if s >= n or t >= n or s == t or (s, t) in seen:
            continue
        seen.add((s, t))
        edges.append((s, t))
    dang = set(perm(n, kd)[:n_dangling])
    pr_ = perm(n, kr)
    kept = sorted((pr_[s], pr_[t]) for s, t in edges if s not in dang)
    rp = np.zeros(n + 1, np.int64)
    for s, _ in kept:
        rp[s + 1] += 1
    return np.cumsum(rp), np.array([t for _, t in kept], np.int32), ctr


def test_rmat_exact_parallel_equals_sequential_definition():
    """The parallel exact-count generator (stable sort of draws, first draw of each edge,
    scan in draw order) returns the same graph as the sequential definition."""
    for n, avg, dfr, seed in ((300, 5.0, 0.1, 3), (1000, 3.0, 0.2, 7), (257, 9.0, 0.05, 11)):
        g = prgen.workload_rmat_n(n, avg, dfr, seed)
        scale = int(np.ceil(np.log2(n)))
        rp, col, draws = _rmat_exact_reference(n, scale, int(round(avg * n)), int(round(dfr * n)), seed,
                                               prgen.WL_RMAT_N)
        assert np.array_equal(g.row_ptr, rp) and np.array_equal(g.col, col), (n, seed)
        assert g.meta["draws"] == draws


def test_batch_and_pool_recipes():
    gs, cs = prgen.workload_batch(count=12, n_lo=1000, n_hi=20000, seed=4)
    assert len(gs) == 12 and set(cs) <= {0.85, 0.9}
    for g in gs:
        _check_csr(g)
        assert 1000 <= g.n <= 20000
        deg = np.diff(g.row_ptr)
        assert (deg == 0).mean() >= 0.05 - 1e-9   # at least the forced dangling share
        assert 3.0 * g.n * 0.75 < g.m <= 32 * g.n
    gs2, cs2 = prgen.workload_batch(count=12, n_lo=1000, n_hi=20000, seed=4, workers=1)
    assert cs2 == cs and all(np.array_equal(a.col, b.col) for a, b in zip(gs, gs2))
    pool = prgen.workload_serve_pool(count=3, n_lo=10_000, n_hi=40_000, seed=2)
    for g in pool:
        _check_csr(g)
        assert 10_000 <= g.n <= 40_000
