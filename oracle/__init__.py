"""CPU oracle for PageRank / PPR and for the IFP1 / IFP2 forward-push algorithms.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library (``paper_2302_03245_amd``) and never imports it.

* ``liboracle.so`` (``oracle.c``, serial FP64): the power method on P'' (Eq. 1),
  serial IFP1 (Algorithm 2) and IFP2 (Algorithm 3) with one calculation thread,
  and a dense Gaussian-elimination solve of Eq. 2 / Eq. 4 for small graphs.
* ``exact`` (pure Python, ``fractions.Fraction``): exact rational solves of Eq. 2
  and Eq. 4 for graphs of a handful of vertices.
* ``weak_dangling_levels`` (numpy): the dangling and weakly dangling vertices of
  section 2, found by deleting dangling vertices round after round.

Every graph argument is any object with ``n``, ``row_ptr`` (int64[n+1]) and
``col`` (int32[m]) attributes, or an ``(n, row_ptr, col)`` tuple.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import exact  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run oracle.build.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_power.restype = ctypes.c_int
    lib.oracle_power.argtypes = [ctypes.c_int64, _I64, _I32, ctypes.c_double, _D, ctypes.c_double,
                                 ctypes.c_int64, _D, _I64, _D]
    lib.oracle_ifp1.restype = ctypes.c_int
    lib.oracle_ifp1.argtypes = [ctypes.c_int64, _I64, _I32, ctypes.c_double, _D, ctypes.c_double,
                                ctypes.c_int64, _D, _D, _D, _I64]
    lib.oracle_ifp2.restype = ctypes.c_int
    lib.oracle_ifp2.argtypes = [ctypes.c_int64, _I64, _I32, ctypes.c_double, _D, ctypes.c_double,
                                ctypes.c_int64, ctypes.c_int, _D, _D, _D, _D, _I64]
    lib.oracle_dense.restype = ctypes.c_int
    lib.oracle_dense.argtypes = [ctypes.c_int64, _I64, _I32, ctypes.c_double, _D, ctypes.c_int, _D]
    _lib = lib
    return lib


def use_library(path: str) -> None:
    """Load the oracle's functions from another build of oracle.c (the host-tuned build
    that times the CPU baseline); later calls use it."""
    global _LIB_PATH, _lib
    _LIB_PATH = path
    _lib = None
    _load()


def _graph(g):
    if isinstance(g, tuple):
        n, rp, col = g
    else:
        n, rp, col = g.n, g.row_ptr, g.col
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(n), rp, col


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _pvec(p, n):
    if p is None:
        return None
    p = np.ascontiguousarray(p, dtype=np.float64)
    if p.shape != (n,):
        raise ValueError("p must have shape (n,)")
    return p


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")
    return rc


def power(g, c: float = 0.85, p=None, tol: float = 1e-13, max_iter: int = 100_000):
    """FP64 power method on P'' until ||x' - x||_1 <= tol; returns (x, iterations, delta).

    The L1 distance of x to the exact PageRank vector is at most c/(1-c) * delta.
    """
    n, rp, col = _graph(g)
    p = _pvec(p, n)
    x = np.empty(n)
    it = ctypes.c_int64(0)
    delta = ctypes.c_double(0)
    rc = _load().oracle_power(n, _ptr(rp, _I64), _ptr(col, _I32), c, _ptr(p, _D), tol, max_iter,
                              _ptr(x, _D), ctypes.byref(it), ctypes.byref(delta))
    _check(rc, "power")
    return x, int(it.value), float(delta.value)


def ifp1(g, c: float = 0.85, p=None, xi: float = 1e-12, max_passes: int = 1_000_000):
    """Serial IFP1; returns dict(pi, pibar, h, passes, vertex_pushes, edge_pushes, converged)."""
    n, rp, col = _graph(g)
    p = _pvec(p, n)
    pi, pb, h = np.empty(n), np.empty(n), np.empty(n)
    counts = np.zeros(3, dtype=np.int64)
    rc = _load().oracle_ifp1(n, _ptr(rp, _I64), _ptr(col, _I32), c, _ptr(p, _D), xi, max_passes,
                             _ptr(pb, _D), _ptr(h, _D), _ptr(pi, _D), _ptr(counts, _I64))
    _check(rc, "ifp1")
    return {"pi": pi, "pibar": pb, "h": h, "passes": int(counts[0]), "vertex_pushes": int(counts[1]),
            "edge_pushes": int(counts[2]), "converged": rc == 0}


def ifp2(g, c: float = 0.85, p=None, xi: float = 1e-12, max_passes: int = 1_000_000, literal: bool = False):
    """Serial IFP2; returns dict(pi, pibar, h, x, passes, vertex_pushes, edge_pushes, phase2_edges, converged)."""
    n, rp, col = _graph(g)
    p = _pvec(p, n)
    pi, pb, h, x = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    counts = np.zeros(4, dtype=np.int64)
    rc = _load().oracle_ifp2(n, _ptr(rp, _I64), _ptr(col, _I32), c, _ptr(p, _D), xi, max_passes,
                             int(bool(literal)), _ptr(pb, _D), _ptr(h, _D), _ptr(x, _D), _ptr(pi, _D),
                             _ptr(counts, _I64))
    _check(rc, "ifp2")
    return {"pi": pi, "pibar": pb, "h": h, "x": x, "passes": int(counts[0]),
            "vertex_pushes": int(counts[1]), "edge_pushes": int(counts[2]),
            "phase2_edges": int(counts[3]), "converged": rc == 0}


def dense(g, c: float = 0.85, p=None, form: int = 0):
    """Dense FP64 solve (n <= 256): form 0 is Eq. 2, form 1 is Eq. 4."""
    n, rp, col = _graph(g)
    p = _pvec(p, n)
    pi = np.empty(n)
    rc = _load().oracle_dense(n, _ptr(rp, _I64), _ptr(col, _I32), c, _ptr(p, _D), form, _ptr(pi, _D))
    _check(rc, "dense")
    return pi


def xi_for_l1(tol: float, c: float, n: int, n_nondangling: int) -> float:
    """Threshold xi for which an emptied frontier certifies an L1 error <= tol.

    With every non-dangling residual <= xi the remaining residual is at most
    n_N * xi, the unnormalised error is at most c/(1-c) times that, the total
    reserved mass is at least n (the initial mass), and normalising at most
    doubles the error.
    """
    return tol * (1.0 - c) / (2.0 * c) * n / max(1, n_nondangling)


def weak_dangling_levels(g, max_levels=None):
    """Deletion round in which each vertex becomes dangling (section 2, graph definitions).

    Round 0 deletes the dangling vertices (no out-edge); round L >= 1 deletes the
    vertices that the earlier deletions left without an out-edge -- the weakly
    dangling vertices.  Returns int64[n]: the round of each vertex, -1 for vertices
    never deleted (they reach a cycle), and for those of rounds above max_levels
    when it is given.  Each round recounts every vertex's out-edges into vertices
    not yet deleted (O(m) per round).
    """
    n, rp, col = _graph(g)
    m = int(rp[n])
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    dst = col[:m].astype(np.int64)
    level = np.full(n, -1, dtype=np.int64)
    deleted = np.zeros(n, dtype=bool)
    rnd = 0
    while max_levels is None or rnd <= max_levels:
        live_out = np.bincount(src[~deleted[dst]], minlength=n)
        new = ~deleted & (live_out == 0)
        if not new.any():
            break
        level[new] = rnd
        deleted |= new
        rnd += 1
    return level
