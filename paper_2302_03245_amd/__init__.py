"""IFP1 / IFP2 forward-push PageRank on an AMD MI355X (gfx950).

Thin ctypes binding of ``libpr.so`` (C ABI in ``include/pr.h``).  Every step of a
solve runs in the library's HIP kernels; this module only marshals arguments.
Host inputs are numpy arrays; device inputs/outputs may be torch CUDA tensors
(passed by pointer, torch is used only for device memory and streams).

    g = upload(row_ptr, col)                       # CSR, int64[n+1], int32[m]
    pi, st = ifp2(g, c=0.85, xi=1e-12)             # numpy float64[n]
    pi, st = ifp2(g, l1_tol=1e-6, residual="fp32", out=torch.empty(n, dtype=torch.float64, device="cuda"))
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpr.so")

PR_OK, PR_ENOCONV, PR_EINVAL, PR_ENOMEM, PR_EDEVICE, PR_EBUSY = 0, 1, -1, -2, -3, -4
PR_RES_FP64, PR_RES_FP32 = 0, 1
PR_STOP_XI, PR_STOP_L1 = 0, 1
PR_INPUT_DEVICE, PR_DEDUPE, PR_PEEL, PR_GROUP_ALL_ROWS = 0x1, 0x2, 0x20000, 0x40000
PR_P_DEVICE, PR_OUT_DEVICE, PR_IFP2_LITERAL = 0x1, 0x2, 0x4
PR_FORCE_PUSH, PR_FORCE_PULL, PR_PROFILE, PR_JACOBI, PR_VERIFY, PR_FORCE_LIST = 0x8, 0x10, 0x20, 0x40, 0x80, 0x100

# every symbol the public headers declare
EXPORTED = ["pr_opts_default", "pr_graph_upload", "pr_graph_free", "pr_graph_info", "pr_solve_ifp1",
            "pr_solve_ifp2", "pr_solve_power", "pr_ppr", "pr_last_error", "pr_last_trace",
            "pr_probe_copy", "pr_probe_gather", "pr_probe_scatter", "pr_probe_gather_out_len",
            "pr_server_opts_default", "pr_server_create", "pr_server_add_graph", "pr_server_footprint", "pr_server_submit",
            "pr_server_wait", "pr_server_get_stats", "pr_server_destroy",
            "pr_set_upload", "pr_set_free", "pr_set_info", "pr_set_solve_ifp2", "pr_set_tune", "pr_graph_tune",
            "pr_state_create", "pr_state_free", "pr_state_read", "pr_solve_ifp2_warm", "pr_state_update",
            "pr_debug_fail_ppr_batch", "pr_solve_ifp2_noalloc"]


class PRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpr status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("xi", ctypes.c_double), ("l1_tol", ctypes.c_double),
                ("stop", ctypes.c_int32), ("residual", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("stream", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("pull_sweeps", ctypes.c_int32),
                ("edges_processed", ctypes.c_int64), ("edges_traversed", ctypes.c_int64),
                ("vertex_pushes", ctypes.c_int64), ("residual_l1", ctypes.c_double),
                ("l1_bound", ctypes.c_double), ("seconds_solve", ctypes.c_double),
                ("seconds_preprocess", ctypes.c_double),
                ("push_seconds", ctypes.c_double), ("push_bytes", ctypes.c_double),
                ("push_launches", ctypes.c_int64),
                ("pull_seconds", ctypes.c_double), ("pull_bytes", ctypes.c_double),
                ("pull_launches", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("l1_verified", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("l1_tol", ctypes.c_double), ("residual", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("batch_min", ctypes.c_int32), ("sweeps_per_round", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("memory_budget", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("edges_per_second", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("graph_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64), ("budget", ctypes.c_int64),
                ("memory_waits", ctypes.c_int64), ("narrowed_runs", ctypes.c_int64), ("rejected", ctypes.c_int64)]


class SetInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n_dangling", ctypes.c_int64), ("m_dangling", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("seconds_upload", ctypes.c_double), ("groups", ctypes.c_int64),
                ("tile_items", ctypes.c_int64), ("ordered", ctypes.c_int64)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("n_dangling", ctypes.c_int64),
                ("m_dangling", ctypes.c_int64), ("n_unreferenced", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("seconds_upload", ctypes.c_double),
                ("seconds_split", ctypes.c_double), ("max_depth", ctypes.c_int64), ("epochs", ctypes.c_int64),
                ("groups", ctypes.c_int64), ("tile_items", ctypes.c_int64), ("ordered", ctypes.c_int64),
                ("n_peeled", ctypes.c_int64), ("peel_levels", ctypes.c_int64)]


class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("tile_shift", ctypes.c_int32 * 16), ("groups", ctypes.c_int32 * 16),
                ("ordered", ctypes.c_int32 * 16), ("ms", ctypes.c_double * 16), ("sweeps", ctypes.c_int32 * 16),
                ("chosen", ctypes.c_int32), ("seconds", ctypes.c_double), ("batch_ordered", ctypes.c_int32),
                ("batch_ms", ctypes.c_double * 2)]


_lib = None


def lib():
    """Load libpr.so; raises if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(the HIP library is required, there is no CPU fallback)")
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname).  Loading
    # torch first makes libpr bind to that copy, so tensors and the library share a runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p
    L.pr_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.pr_opts_default.restype = None
    L.pr_graph_upload.argtypes = [i64, i64, vp, vp, u32, ctypes.POINTER(vp)]
    L.pr_graph_upload.restype = ctypes.c_int
    L.pr_graph_free.argtypes = [vp]
    L.pr_graph_free.restype = ctypes.c_int
    L.pr_graph_info.argtypes = [vp, ctypes.POINTER(GraphInfo)]
    L.pr_graph_info.restype = ctypes.c_int
    for name in ("pr_solve_ifp1", "pr_solve_ifp2", "pr_solve_power"):
        f = getattr(L, name)
        f.argtypes = [vp, dp, ctypes.POINTER(Opts), dp, ctypes.POINTER(Stats)]
        f.restype = ctypes.c_int
    L.pr_ppr.argtypes = [vp, vp, i32, ctypes.POINTER(Opts), dp, ctypes.POINTER(Stats)]
    L.pr_ppr.restype = ctypes.c_int
    L.pr_last_error.argtypes = []
    L.pr_last_error.restype = ctypes.c_char_p
    L.pr_last_trace.argtypes = [i32, vp, vp, vp, vp, vp]
    L.pr_last_trace.restype = i32
    L.pr_probe_copy.argtypes = [vp, vp, i64, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double)]
    L.pr_probe_copy.restype = ctypes.c_int
    L.pr_probe_gather.argtypes = [vp, vp, i64, vp, i64, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double)]
    L.pr_probe_gather.restype = ctypes.c_int
    L.pr_probe_scatter.argtypes = [vp, vp, i64, ctypes.c_float, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double)]
    L.pr_probe_scatter.restype = ctypes.c_int
    L.pr_probe_gather_out_len.argtypes = [i64]
    L.pr_probe_gather_out_len.restype = i64
    L.pr_state_create.argtypes = [i64, vp, ctypes.POINTER(vp)]
    L.pr_state_create.restype = ctypes.c_int
    L.pr_state_free.argtypes = [vp]
    L.pr_state_free.restype = ctypes.c_int
    L.pr_state_read.argtypes = [vp, vp, vp]
    L.pr_state_read.restype = ctypes.c_int
    L.pr_solve_ifp2_warm.argtypes = [vp, ctypes.POINTER(Opts), vp, dp, ctypes.POINTER(Stats)]
    L.pr_solve_ifp2_warm.restype = ctypes.c_int
    L.pr_state_update.argtypes = [vp, vp, vp, vp, i32]
    L.pr_state_update.restype = ctypes.c_int
    L.pr_graph_tune.argtypes = [vp, ctypes.POINTER(Opts), i32, ctypes.POINTER(TuneReport)]
    L.pr_graph_tune.restype = ctypes.c_int
    L.pr_set_upload.argtypes = [i32, vp, vp, vp, u32, ctypes.POINTER(vp)]
    L.pr_set_upload.restype = ctypes.c_int
    L.pr_set_free.argtypes = [vp]
    L.pr_set_free.restype = ctypes.c_int
    L.pr_set_info.argtypes = [vp, ctypes.POINTER(SetInfo)]
    L.pr_set_info.restype = ctypes.c_int
    L.pr_set_solve_ifp2.argtypes = [vp, vp, ctypes.POINTER(Opts), dp, ctypes.POINTER(Stats)]
    L.pr_set_solve_ifp2.restype = ctypes.c_int
    L.pr_set_tune.argtypes = [vp, vp, ctypes.POINTER(Opts), i32, ctypes.POINTER(TuneReport)]
    L.pr_set_tune.restype = ctypes.c_int
    L.pr_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    L.pr_server_opts_default.restype = None
    L.pr_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.pr_server_create.restype = ctypes.c_int
    L.pr_server_add_graph.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.pr_server_add_graph.restype = ctypes.c_int
    L.pr_server_submit.argtypes = [vp, i32, i32, vp, ctypes.POINTER(i64)]
    L.pr_server_submit.restype = ctypes.c_int
    L.pr_server_wait.argtypes = [vp, i64, ctypes.c_double, ctypes.POINTER(Stats)]
    L.pr_server_wait.restype = ctypes.c_int
    L.pr_server_footprint.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_int64)]
    L.pr_server_footprint.restype = ctypes.c_int
    L.pr_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.pr_server_get_stats.restype = ctypes.c_int
    L.pr_server_destroy.argtypes = [vp]
    L.pr_server_destroy.restype = ctypes.c_int
    L.pr_debug_fail_ppr_batch.argtypes = [i32]
    L.pr_debug_fail_ppr_batch.restype = None
    L.pr_solve_ifp2_noalloc.argtypes = [vp, dp, ctypes.POINTER(Opts), dp, ctypes.POINTER(Stats)]
    L.pr_solve_ifp2_noalloc.restype = ctypes.c_int
    _lib = L
    return L


def _err(status):
    return PRError(status, lib().pr_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr_host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _ptr_any(x, np_dtype, torch_dtype_name):
    """(keepalive, pointer, on_device) for a numpy array or a torch tensor."""
    if x is None:
        return None, None, False
    if _is_torch(x):
        if str(x.dtype) != f"torch.{torch_dtype_name}":
            raise TypeError(f"expected a {torch_dtype_name} tensor")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x, x.data_ptr(), x.is_cuda
    a, p = _ptr_host(x, np_dtype)
    return a, p, False


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Graph:
    """A graph resident in device memory (handle of pr_graph_upload)."""

    def __init__(self, handle, n, m):
        self._h = handle
        self.n, self.m = n, m

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph was freed")
        return self._h

    def info(self) -> dict:
        gi = GraphInfo()
        st = lib().pr_graph_info(self.handle, ctypes.byref(gi))
        if st != PR_OK:
            raise _err(st)
        return {k: getattr(gi, k) for k, _ in gi._fields_}

    def free(self):
        if self._h is not None:
            lib().pr_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def upload(row_ptr, col, dedupe: bool = False, tile_shift: int = 0, groups: int = 0, sort_in: bool = True,
           peel: bool = False, group_rows: bool = True) -> Graph:
    """Copy a CSR graph (host numpy or device torch tensors) to the device.

    `tile_shift` s in {2, 3, 4} sets 256 << s rows + edges per sweep tile (0: default);
    `groups` k in 1..15 sets the vertex groups of ordered sweeps (0: 4 on graphs with at least
    2^24 edges between non-dangling vertices, else none; 1: none); `peel` takes weakly
    dangling vertices out of IFP2's sweeps (PR_PEEL: IFP2 and PPR only); `group_rows`
    False makes each group's gather walk every row (PR_GROUP_ALL_ROWS)."""
    rp_keep, rp_ptr, rp_dev = _ptr_any(row_ptr, np.int64, "int64")
    col_keep, col_ptr, col_dev = _ptr_any(col, np.int32, "int32")
    if rp_dev != col_dev:
        raise ValueError("row_ptr and col must both be host or both be device buffers")
    n = (rp_keep.shape[0] if not _is_torch(rp_keep) else rp_keep.numel()) - 1
    m = col_keep.shape[0] if not _is_torch(col_keep) else col_keep.numel()
    flags = (PR_INPUT_DEVICE if rp_dev else 0) | (PR_DEDUPE if dedupe else 0) | ((tile_shift & 7) << 8) | \
        ((groups & 15) << 12) | (0 if sort_in else 0x10000) | (PR_PEEL if peel else 0) | \
        (0 if group_rows else PR_GROUP_ALL_ROWS)
    h = ctypes.c_void_p()
    st = lib().pr_graph_upload(int(n), int(m), rp_ptr, col_ptr if m else None, flags, ctypes.byref(h))
    if st != PR_OK:
        raise _err(st)
    g = Graph(h.value, int(n), int(m))
    if dedupe:
        g.m = g.info()["m"]
    return g


def tune(g: Graph, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", reps=2) -> dict:
    """Autotune the sweep schedule of global solves on g (pr_graph_tune); returns the report."""
    o = _opts(c, xi, l1_tol, residual, 0, None, False, None, False)
    r = TuneReport()
    st = lib().pr_graph_tune(g.handle, ctypes.byref(o), int(reps), ctypes.byref(r))
    if st != PR_OK:
        raise _err(st)
    k = r.candidates
    cands = [{"tile_shift": r.tile_shift[i], "ordered": bool(r.ordered[i]), "group_rows": r.ordered[i] == 2,
              "groups": r.groups[i], "ms": r.ms[i], "sweeps": r.sweeps[i]} for i in range(k)]
    return {"candidates": cands, "chosen": cands[r.chosen], "seconds": r.seconds,
            "batch_ordered": r.batch_ordered, "batch_ms": {"ordered": r.batch_ms[0], "synchronous": r.batch_ms[1]}}


class State:
    """Reserve and residual of a forward-push solve, carried across graph changes
    (include/pr_warm.h).  p: host personalisation (None: uniform), used for the cold start."""

    def __init__(self, n: int, p=None):
        self.n = int(n)
        pk = None if p is None else np.ascontiguousarray(p, dtype=np.float64)
        if pk is not None and pk.shape != (self.n,):
            raise ValueError("p must have n entries")
        h = ctypes.c_void_p()
        st = lib().pr_state_create(self.n, pk.ctypes.data if pk is not None else None, ctypes.byref(h))
        if st != PR_OK:
            raise _err(st)
        self._h = h.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("state was freed")
        return self._h

    def read(self):
        pb, h = np.empty(self.n), np.empty(self.n)
        st = lib().pr_state_read(self.handle, pb.ctypes.data, h.ctypes.data)
        if st != PR_OK:
            raise _err(st)
        return pb, h

    def update(self, g_old: Graph, g_new: Graph, changed=None):
        """h += c (P_new - P_old) pibar over the changed sources (all when None)."""
        ch = None if changed is None else np.ascontiguousarray(changed, dtype=np.int32)
        st = lib().pr_state_update(self.handle, g_old.handle, g_new.handle,
                                   ch.ctypes.data if ch is not None and ch.size else None,
                                   0 if ch is None else int(ch.size))
        if st != PR_OK:
            raise _err(st)

    def free(self):
        if self._h is not None:
            lib().pr_state_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ifp2_warm(g: Graph, state: State, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, out=None,
              stream=None, mode=None, profile=False, verify=False):
    """IFP2 resumed from `state` (and leaving its end state there)."""
    o = _opts(c, xi, l1_tol, residual, max_sweeps, stream, False, mode, profile, verify=verify)
    if out is None:
        out = np.empty(g.n, dtype=np.float64)
    out_keep, out_ptr, out_dev = _ptr_any(out, np.float64, "float64")
    if (out_keep.numel() if _is_torch(out_keep) else out_keep.shape[0]) != g.n:
        raise ValueError("out must have n entries")
    if not _is_torch(out) and out_keep is not out:
        raise ValueError("out must be a contiguous float64 numpy array")
    if out_dev:
        o.flags |= PR_OUT_DEVICE
    st = Stats()
    status = lib().pr_solve_ifp2_warm(g.handle, ctypes.byref(o), state.handle, out_ptr, ctypes.byref(st))
    if status < 0:
        raise _err(status)
    return out, dict(st.as_dict(), status=status)


class GraphSet:
    """k graphs resident in device memory as one union (handle of pr_set_upload)."""

    def __init__(self, handle, sizes):
        self._h = handle
        self.sizes = [int(x) for x in sizes]
        self.k = len(self.sizes)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph set was freed")
        return self._h

    def info(self) -> dict:
        si = SetInfo()
        st = lib().pr_set_info(self.handle, ctypes.byref(si))
        if st != PR_OK:
            raise _err(st)
        return {k: getattr(si, k) for k, _ in si._fields_}

    def split(self, pi):
        """Per-graph views of a solution over the whole set."""
        return [pi[int(self.offsets[g]):int(self.offsets[g + 1])] for g in range(self.k)]

    def free(self):
        if self._h is not None:
            lib().pr_set_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def upload_set(graphs, tile_shift: int = 0, groups: int = 0) -> GraphSet:
    """Upload host CSR graphs [(row_ptr int64[n+1], col int32[m]), ...] as one graph set.
    `groups` q in 1..15: vertex groups per graph for ordered sweeps (0: 4; 1: none)."""
    k = len(graphs)
    rps = [np.ascontiguousarray(rp, dtype=np.int64) for rp, _ in graphs]
    cols = [np.ascontiguousarray(c, dtype=np.int32) for _, c in graphs]
    ns = np.array([r.shape[0] - 1 for r in rps], dtype=np.int64)
    rp_ptrs = (ctypes.c_void_p * max(k, 1))(*[r.ctypes.data for r in rps])
    col_ptrs = (ctypes.c_void_p * max(k, 1))(*[c.ctypes.data if c.size else None for c in cols])
    h = ctypes.c_void_p()
    st = lib().pr_set_upload(k, ns.ctypes.data if k else None, rp_ptrs, col_ptrs,
                             ((tile_shift & 7) << 8) | ((groups & 15) << 12), ctypes.byref(h))
    if st != PR_OK:
        raise _err(st)
    return GraphSet(h.value, ns)


def set_ifp2(gs: GraphSet, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, out=None, stream=None,
             mode=None, jacobi=False):
    """IFP2 on every graph of a set: c is one factor or one per graph; `jacobi` keeps
    synchronous sweeps on a set with vertex groups.  Returns (solution over the whole
    set, list of per-graph stats dicts)."""
    o = _opts(0.85, xi, l1_tol, residual, max_sweeps, stream, False, mode, False, jacobi=jacobi)
    cs = None
    if np.ndim(c) == 0:
        o.c = float(c)
    else:
        cs = np.ascontiguousarray(c, dtype=np.float64)
        if cs.shape != (gs.k,):
            raise ValueError("c must be a scalar or have one entry per graph")
    if out is None:
        out = np.empty(gs.n, dtype=np.float64)
    out_keep, out_ptr, out_dev = _ptr_any(out, np.float64, "float64")
    if (out_keep.numel() if _is_torch(out_keep) else out_keep.shape[0]) != gs.n:
        raise ValueError("out must have one entry per vertex of the set")
    if not _is_torch(out) and out_keep is not out:
        raise ValueError("out must be a contiguous float64 numpy array")
    if out_dev:
        o.flags |= PR_OUT_DEVICE
    st = (Stats * gs.k)()
    status = lib().pr_set_solve_ifp2(gs.handle, cs.ctypes.data if cs is not None else None, ctypes.byref(o),
                                     out_ptr, st)
    if status < 0:
        raise _err(status)
    return out, [dict(st[i].as_dict(), status=status) for i in range(gs.k)]


def set_tune(gs: GraphSet, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", reps=2) -> dict:
    """Autotune the sweep schedule of set solves (pr_set_tune); returns the report."""
    o = _opts(0.85, xi, l1_tol, residual, 0, None, False, None, False)
    cs = None
    if np.ndim(c) == 0:
        o.c = float(c)
    else:
        cs = np.ascontiguousarray(c, dtype=np.float64)
        if cs.shape != (gs.k,):
            raise ValueError("c must be a scalar or have one entry per graph")
    r = TuneReport()
    st = lib().pr_set_tune(gs.handle, cs.ctypes.data if cs is not None else None, ctypes.byref(o), int(reps),
                           ctypes.byref(r))
    if st != PR_OK:
        raise _err(st)
    cands = [{"tile_shift": r.tile_shift[i], "ordered": bool(r.ordered[i]), "groups": r.groups[i], "ms": r.ms[i],
              "sweeps": r.sweeps[i]} for i in range(r.candidates)]
    return {"candidates": cands, "chosen": cands[r.chosen], "seconds": r.seconds}


def _opts(c, xi, l1_tol, residual, max_sweeps, stream, literal, mode, profile, power=False, jacobi=False,
          verify=False):
    o = Opts()
    lib().pr_opts_default(ctypes.byref(o))
    o.c = c
    if xi is not None:
        o.xi = xi
    if l1_tol is not None:
        o.l1_tol = l1_tol
        if not power:
            o.stop = PR_STOP_L1
    o.residual = {"fp64": PR_RES_FP64, "fp32": PR_RES_FP32}[residual]
    o.max_sweeps = max_sweeps
    o.stream = _stream_handle(stream)
    flags = 0
    if literal:
        flags |= PR_IFP2_LITERAL
    if mode == "push":
        flags |= PR_FORCE_PUSH
    elif mode == "pull":
        flags |= PR_FORCE_PULL
    elif mode == "list":
        flags |= PR_FORCE_LIST
    elif mode is not None:
        raise ValueError("mode must be None, 'push', 'pull' or 'list'")
    if profile:
        flags |= PR_PROFILE
    if jacobi:
        flags |= PR_JACOBI
    if verify:
        flags |= PR_VERIFY
    o.flags = flags
    return o


def _solve(fn, g, p, o, out):
    p_keep, p_ptr, p_dev = _ptr_any(p, np.float64, "float64")
    if p is not None:
        n_p = p_keep.numel() if _is_torch(p_keep) else p_keep.shape[0]
        if n_p != g.n:
            raise ValueError("p must have n entries")
    if p_dev:
        o.flags |= PR_P_DEVICE
    if out is None:
        out = np.empty(g.n, dtype=np.float64)
    out_keep, out_ptr, out_dev = _ptr_any(out, np.float64, "float64")
    if (out_keep.numel() if _is_torch(out_keep) else out_keep.shape[0]) != g.n:
        raise ValueError("out must have n entries")
    if not _is_torch(out) and out_keep is not out:
        raise ValueError("out must be a contiguous float64 numpy array")
    if out_dev:
        o.flags |= PR_OUT_DEVICE
    st = Stats()
    status = fn(g.handle, p_ptr, ctypes.byref(o), out_ptr, ctypes.byref(st))
    if status < 0:
        raise _err(status)
    d = st.as_dict()
    d["status"] = status
    return out, d


def ifp1(g: Graph, p=None, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, out=None,
         stream=None, mode=None, profile=False, jacobi=False, verify=False):
    """IFP1 (Algorithm 2).  `l1_tol` switches to the certified-L1 stop rule; `jacobi`
    keeps synchronous sweeps on a graph with vertex groups; `verify` adds the
    a-posteriori bound l1_verified (PR_VERIFY)."""
    o = _opts(c, xi, l1_tol, residual, max_sweeps, stream, False, mode, profile, jacobi=jacobi, verify=verify)
    return _solve(lib().pr_solve_ifp1, g, p, o, out)


def ifp2(g: Graph, p=None, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, out=None,
         stream=None, literal=False, mode=None, profile=False, jacobi=False, verify=False):
    """IFP2 (Algorithm 3).  `literal` drops the leftover residual at normalisation;
    `jacobi` keeps global solves on synchronous sweeps (no ordered groups); `verify`
    adds the a-posteriori bound l1_verified (PR_VERIFY)."""
    o = _opts(c, xi, l1_tol, residual, max_sweeps, stream, literal, mode, profile, jacobi=jacobi, verify=verify)
    return _solve(lib().pr_solve_ifp2, g, p, o, out)


def ifp2_noalloc(g: Graph, p=None, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, out=None,
                 stream=None, literal=False, mode=None, jacobi=False, verify=False):
    """IFP2 through pr_solve_ifp2_noalloc: the workspace comes from the library's fixed
    device array (no allocation in the call); otherwise as ifp2()."""
    o = _opts(c, xi, l1_tol, residual, max_sweeps, stream, literal, mode, False, jacobi=jacobi, verify=verify)
    return _solve(lib().pr_solve_ifp2_noalloc, g, p, o, out)


def power(g: Graph, p=None, c=0.85, l1_tol=1e-9, residual="fp64", max_sweeps=0, out=None, stream=None,
          profile=False, verify=False):
    """Power method on P'' until the certified L1 error is <= l1_tol."""
    o = _opts(c, None, l1_tol, residual, max_sweeps, stream, False, None, profile, power=True, verify=verify)
    return _solve(lib().pr_solve_power, g, p, o, out)


def last_trace() -> dict:
    """Per-sweep record of this thread's last profiled IFP solve (see pr_last_trace)."""
    L = lib()
    n = L.pr_last_trace(0, None, None, None, None, None)
    active, edges = np.zeros(n, np.int64), np.zeros(n, np.int64)
    residual, bound = np.zeros(n), np.zeros(n)
    pulled = np.zeros(n, np.int32)
    if n:
        L.pr_last_trace(n, active.ctypes.data, edges.ctypes.data, residual.ctypes.data, bound.ctypes.data,
                        pulled.ctypes.data)
    return {"active": active, "edges": edges, "residual": residual, "bound": bound, "pulled": pulled}


def ppr(g: Graph, sources, c=0.85, xi=1e-12, l1_tol=None, residual="fp64", max_sweeps=0, stream=None,
        mode=None, out=None, jacobi=False, verify=False):
    """Single-source PPR for each source (IFP2, sources batched sixteen at a time);
    returns (float64[k, n], list of stats dicts).  `out` may be a (k, n) float64 numpy
    array or torch CUDA tensor."""
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    o = _opts(c, xi, l1_tol, residual, max_sweeps, stream, False, mode, False, jacobi=jacobi, verify=verify)
    if out is None:
        out = np.empty((k, g.n), dtype=np.float64)
    out_keep, out_ptr, out_dev = _ptr_any(out, np.float64, "float64")
    size = out_keep.numel() if _is_torch(out_keep) else out_keep.size
    if size != k * g.n or (not _is_torch(out) and out_keep is not out):
        raise ValueError("out must be a contiguous float64 array of k * n entries")
    if out_dev:
        o.flags |= PR_OUT_DEVICE
    st = (Stats * max(k, 1))()
    status = lib().pr_ppr(g.handle, src.ctypes.data if k else None, k, ctypes.byref(o), out_ptr, st)
    if status < 0:
        raise _err(status)
    return out, [dict(st[i].as_dict(), status=status) for i in range(k)]


def debug_fail_ppr_batch(b):
    """Testing hook: the next ppr() call on this thread fails with PR_ENOMEM on reaching
    batch b (after b batches of sixteen sources were solved); b <= 0 disables it."""
    lib().pr_debug_fail_ppr_batch(int(b))


class Server:
    """Query server over resident graphs (include/pr_serve.h): global PageRank and
    single-source PPR queries, solved alone when an engine's queue is short and
    continuously batched otherwise, engines overlapping on the device.  Results are
    written into caller-owned torch CUDA float64 tensors."""

    def __init__(self, c=0.85, l1_tol=1e-6, residual="fp32", slots=16, sweeps_per_round=4, max_sweeps=0,
                 memory_budget=0, batch_min=2):
        L = lib()
        o = ServerOpts()
        L.pr_server_opts_default(ctypes.byref(o))
        o.c, o.l1_tol = c, l1_tol
        o.residual = {"fp64": PR_RES_FP64, "fp32": PR_RES_FP32}[residual]
        o.slots, o.sweeps_per_round, o.max_sweeps, o.memory_budget = slots, sweeps_per_round, max_sweeps, memory_budget
        o.batch_min = batch_min
        h = ctypes.c_void_p()
        st = L.pr_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != PR_OK:
            raise _err(st)
        self._h = h.value
        self._graphs = []   # keep the graphs alive while the server runs
        self._outs = {}

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        st = lib().pr_server_add_graph(self._h, g.handle, ctypes.byref(gid))
        if st != PR_OK:
            raise _err(st)
        self._graphs.append(g)
        return gid.value

    def footprint(self, graph_id: int, width: int) -> int:
        """Device bytes of a run's workspace on a registered graph: width 1 (one query
        solved alone), 8 or 16 (a batched run of that many query slots)."""
        b = ctypes.c_int64()
        st = lib().pr_server_footprint(self._h, graph_id, width, ctypes.byref(b))
        if st != PR_OK:
            raise _err(st)
        return b.value

    def submit(self, graph_id: int, source: int, out) -> int:
        """source = -1: global PageRank; out: contiguous torch CUDA float64 tensor of n entries."""
        if not (_is_torch(out) and out.is_cuda and str(out.dtype) == "torch.float64" and out.is_contiguous()):
            raise TypeError("out must be a contiguous CUDA float64 tensor")
        rid = ctypes.c_int64()
        st = lib().pr_server_submit(self._h, graph_id, source, out.data_ptr(), ctypes.byref(rid))
        if st != PR_OK:
            raise _err(st)
        self._outs[rid.value] = out
        return rid.value

    def wait(self, request_id: int, timeout: float = -1.0) -> dict:
        s = Stats()
        st = lib().pr_server_wait(self._h, request_id, timeout, ctypes.byref(s))
        self._outs.pop(request_id, None)
        if st < 0:
            raise _err(st)
        d = s.as_dict()
        d["status"] = st
        return d

    def stats(self) -> dict:
        s = ServerStats()
        st = lib().pr_server_get_stats(self._h, ctypes.byref(s))
        if st != PR_OK:
            raise _err(st)
        return {k: getattr(s, k) for k, _ in s._fields_}

    def close(self):
        if self._h is not None:
            lib().pr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
