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
