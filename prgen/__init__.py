"""Seeded synthetic graph generators shared by the GPU tests, the bench and the oracle tests.

This package only produces inputs: directed graphs as CSR arrays
(``row_ptr`` int64[n+1], ``col`` int32[m], each row sorted by target) and
personalization vectors.  It holds none of the PageRank arithmetic.

The large recipes run in ``libprgen.so`` (C + OpenMP, counter-based SplitMix64
streams, identical output for any thread count); the tiny test graphs are drawn
with numpy's seeded ``default_rng``.

Workload recipes (the paper's six public graphs are not available; these stand in
for them with the same kinds of structure, see the experiment section of the paper):

* ``workload_rmat_small``: R-MAT a/b/c/d = .57/.19/.19/.05 drawn at scale 14,
  endpoints >= 10,000 rejected, self-loops and repeats dropped, drawn until
  100,000 distinct edges exist; then all out-edges of 1,000 uniformly chosen
  vertices (10 %) are dropped.  Seed 0.
* ``workload_rmat(scale=22)``: 16 * 2**22 R-MAT draws, self-loops and repeats
  removed; out-edges of a random 15 % of vertices dropped; edges into a further
  random 10 % redirected to uniform vertices outside that set.
* ``workload_dag``: 2**23 vertices in 64 random layers, Zipf(2.0) out-degrees
  capped at 10,000 and scaled to 80M forward edges, plus 2 % back edges.
* ``workload_rmat_n``: R-MAT at any n (drawn at scale ceil(log2 n), endpoints
  >= n rejected) with an exact number of distinct edges avg_degree * n, then
  the out-edges of a random dangling_frac of the vertices dropped.
* ``workload_batch``: many independent ``workload_rmat_n`` graphs, n
  log-uniform in [1k, 500k], average degree uniform in [4, 32], 5-20 % dangling,
  damping factor drawn from {0.85, 0.9} per graph.
* ``workload_serve_pool``: a resident pool of ``workload_rmat_n`` graphs with n
  log-uniform in [10k, 4M], average degree 16, 15 % dangling.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libprgen.so")
_lib = None


class _CGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("aux", ctypes.c_double),
        ("draws", ctypes.c_int64),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() or prgen.build.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_CGraph)
    lib.prgen_rmat_exact.restype = P
    lib.prgen_rmat_exact.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_uint32]
    lib.prgen_rmat.restype = P
    lib.prgen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64, ctypes.c_uint32]
    lib.prgen_dag.restype = P
    lib.prgen_dag.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32]
    lib.prgen_free.restype = None
    lib.prgen_free.argtypes = [P]
    _lib = lib
    return lib


@dataclass
class Graph:
    """A directed graph in CSR form: edges i -> col[row_ptr[i]:row_ptr[i+1]]."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])


def _take(res, name, meta) -> Graph:
    if not res:
        raise ValueError(f"generator rejected the parameters of {name}")
    r = res.contents
    n, m = int(r.n), int(r.m)
    rp = np.ctypeslib.as_array(r.row_ptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(r.col, shape=(max(m, 1),))[:m].copy()
    meta = dict(meta)
    meta["draws"] = int(r.draws)
    if name.startswith("dag"):
        meta["lambda"] = float(r.aux)
    _load().prgen_free(res)
    return Graph(n=n, row_ptr=rp, col=col, name=name, meta=meta)


def _cache_path(key: str):
    d = os.environ.get("PRGEN_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, hashlib.sha1(key.encode()).hexdigest()[:16] + ".npz")


def _cached(key: str, make):
    path = _cache_path(key)
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Graph(n=int(z["n"]), row_ptr=z["row_ptr"], col=z["col"], name=str(z["name"]),
                     meta={"draws": int(z["draws"]), "lambda": float(z["lam"])})
    g = make()
    if path:
        np.savez(path, n=g.n, row_ptr=g.row_ptr, col=g.col, name=g.name,
                 draws=g.meta.get("draws", 0), lam=g.meta.get("lambda", 0.0))
    return g


# workload ids keep the random streams of different recipes independent
WL_RMAT_SMALL, WL_RMAT, WL_DAG, WL_RMAT_N = 1, 2, 3, 4


def workload_rmat_small(seed: int = 0, n: int = 10_000, scale: int = 14, m: int = 100_000,
                        n_dangling: int = 1_000, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT with n=10,000 and 100,000 distinct edges, 10 % of vertices made dangling."""
    lib = _load()
    res = lib.prgen_rmat_exact(n, scale, m, n_dangling, a, b, c, seed, WL_RMAT_SMALL)
    return _take(res, f"rmat_small_n{n}_m{m}_s{seed}", {"seed": seed})


def workload_rmat(scale: int = 22, edge_factor: int = 16, dangling_frac: float = 0.15,
                  unref_frac: float = 0.10, seed: int = 0, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT at `scale` with `edge_factor` draws per vertex, dangling / unreferenced transforms."""
    key = f"rmat:{scale}:{edge_factor}:{dangling_frac}:{unref_frac}:{seed}:{a}:{b}:{c}"

    def make():
        res = _load().prgen_rmat(scale, edge_factor, a, b, c, dangling_frac, unref_frac, seed, WL_RMAT)
        return _take(res, f"rmat_scale{scale}_ef{edge_factor}_s{seed}", {"seed": seed})
    return _cached(key, make)


def workload_dag(n_layers: int = 64, layer_size: int = 131_072, zipf_s: float = 2.0,
                 zmax: int = 10_000, target_edges: int = 80_000_000, back_frac: float = 0.02,
                 seed: int = 0) -> Graph:
    """Layered DAG with Zipf out-degrees and a small fraction of back edges."""
    key = f"dag:{n_layers}:{layer_size}:{zipf_s}:{zmax}:{target_edges}:{back_frac}:{seed}"

    def make():
        res = _load().prgen_dag(n_layers, layer_size, zipf_s, zmax, target_edges, back_frac, seed, WL_DAG)
        return _take(res, f"dag_L{n_layers}_w{layer_size}_s{seed}", {"seed": seed})
    return _cached(key, make)


def workload_rmat_n(n: int, avg_degree: float, dangling_frac: float, seed: int,
                    a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT with any n: drawn at scale ceil(log2 n), endpoints >= n, self-loops and
    repeats rejected until round(avg_degree * n) distinct edges exist; then all
    out-edges of round(dangling_frac * n) uniformly chosen vertices are dropped."""
    scale = max(1, int(np.ceil(np.log2(max(n, 2)))))
    m = int(round(avg_degree * n))
    nd = int(round(dangling_frac * n))
    key = f"rmatn:{n}:{m}:{nd}:{seed}:{a}:{b}:{c}"

    def make():
        res = _load().prgen_rmat_exact(n, scale, m, nd, a, b, c, seed, WL_RMAT_N)
        return _take(res, f"rmatn_n{n}_m{m}_s{seed}", {"seed": seed})
    return _cached(key, make)


def _many(params, workers):
    """Generate several workload_rmat_n graphs on a thread pool (the C calls run
    without the GIL); the result does not depend on the worker count."""
    from concurrent.futures import ThreadPoolExecutor
    if workers is None:
        workers = min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(lambda q: workload_rmat_n(*q), params))


def workload_batch(count: int = 256, n_lo: int = 1_000, n_hi: int = 500_000, deg_lo: float = 4.0,
                   deg_hi: float = 32.0, dangling_lo: float = 0.05, dangling_hi: float = 0.20,
                   c_choices=(0.85, 0.9), seed: int = 0, workers=None):
    """Independent graphs for batched solves: returns (graphs, c per graph)."""
    rng = np.random.default_rng([seed, WL_RMAT_N, 100])
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).round().astype(np.int64)
    degs = rng.uniform(deg_lo, deg_hi, count)
    dfr = rng.uniform(dangling_lo, dangling_hi, count)
    cs = rng.choice(np.asarray(c_choices, dtype=np.float64), count)
    params = [(int(ns[i]), float(degs[i]), float(dfr[i]), seed * 100_003 + i) for i in range(count)]
    return _many(params, workers), [float(x) for x in cs]


def workload_serve_pool(count: int = 32, n_lo: int = 10_000, n_hi: int = 4_000_000,
                        avg_degree: float = 16.0, dangling_frac: float = 0.15, seed: int = 0, workers=None):
    """Resident graphs answering global PageRank queries in the served scenario."""
    rng = np.random.default_rng([seed, WL_RMAT_N, 200])
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).round().astype(np.int64)
    params = [(int(ns[i]), avg_degree, dangling_frac, seed * 100_003 + 50_000 + i) for i in range(count)]
    return _many(params, workers)


def from_edges(n: int, src, dst, name: str = "") -> Graph:
    """CSR from an edge list (kept in the given multiplicity; rows sorted by target)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return Graph(n=n, row_ptr=rp.astype(np.int64), col=dst.astype(np.int32), name=name)


def random_digraph(n: int, m: int, seed: int, self_loops: bool = False, multi: bool = False,
                   dangling_frac: float = 0.0, unref_frac: float = 0.0) -> Graph:
    """Small seeded random digraph (numpy), for tests.

    Draws m (src, dst) pairs uniformly; unless `multi`, repeats are removed; unless
    `self_loops`, self-loops are removed.  Then the out-edges of a random
    `dangling_frac` of vertices are dropped and the in-edges of a further random
    `unref_frac` are dropped.
    """
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=m)
    d = rng.integers(0, n, size=m)
    if not self_loops:
        keep = s != d
        s, d = s[keep], d[keep]
    if not multi and len(s):
        key = np.unique(s * n + d)
        s, d = key // n, key % n
    perm = rng.permutation(n)
    nd = int(dangling_frac * n)
    nu = int(unref_frac * n)
    dang = np.zeros(n, bool)
    dang[perm[:nd]] = True
    unref = np.zeros(n, bool)
    unref[perm[nd:nd + nu]] = True
    keep = ~dang[s] & ~unref[d]
    return from_edges(n, s[keep], d[keep], name=f"random_n{n}_m{m}_s{seed}")


def uniform_p(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n)


def random_p(n: int, seed: int, zero_frac: float = 0.0) -> np.ndarray:
    """A seeded personalization vector (nonnegative, sums to 1, optional zeros)."""
    rng = np.random.default_rng(seed)
    p = rng.random(n)
    if zero_frac > 0:
        p[rng.random(n) < zero_frac] = 0.0
        if p.sum() == 0:
            p[0] = 1.0
    return p / p.sum()


def stats(g: Graph) -> dict:
    """The columns of the paper's data-set table for a generated graph, plus skew figures."""
    deg = np.diff(g.row_ptr)
    indeg = np.bincount(g.col, minlength=g.n) if g.m else np.zeros(g.n, np.int64)
    dang = deg == 0
    m_d = int(dang[g.col].sum()) if g.m else 0
    return {
        "n": g.n, "m": g.m, "n_d": int(dang.sum()), "m_d": m_d,
        "n_u": int((indeg == 0).sum()), "deg": g.m / g.n,
        "max_out": int(deg.max()) if g.n else 0, "max_in": int(indeg.max()) if g.n else 0,
    }
