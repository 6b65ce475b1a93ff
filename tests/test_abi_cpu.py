"""The C ABI library without a GPU: it loads, exports every symbol the public
headers declare, and rejects invalid host arguments before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2302_03245_amd", "libpr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libpr.so not built")


def _declared():
    names = set()
    for h in ("pr.h", "pr_probe.h", "pr_serve.h", "pr_set.h", "pr_warm.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w \*]*?\b(pr_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    import paper_2302_03245_amd as pr

    names = _declared()
    assert len(names) >= 31
    lib = ctypes.CDLL(LIB)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pr.EXPORTED)


def test_opts_default():
    import paper_2302_03245_amd as pr

    o = pr.Opts()
    pr.lib().pr_opts_default(ctypes.byref(o))
    assert o.c == 0.85 and o.xi == 1e-12 and o.l1_tol == 1e-6
    assert o.stop == pr.PR_STOP_XI and o.residual == pr.PR_RES_FP64 and o.flags == 0


@pytest.mark.parametrize("n,m,rp,col,flags,msg", [
    (0, 0, [0], [], 0, "n must be"),
    (3, 2, [0, 1, 1, 2], [1, 2], 0x80, "unknown upload flag"),
    (3, 1, [1, 1, 1, 2], [1], 0, "row_ptr[0]"),
    (3, 2, [0, 2, 1, 2], [1, 2], 0, "non-decreasing"),
    (3, 2, [0, 1, 1, 3], [1, 2], 0, "row_ptr[n] != m"),
    (3, -1, [0, 1, 1, 2], [1, 2], 0, "m must be"),
    (3, 2, [0, 1, 1, 2], [1, 7], 0x2, "out of [0, n)"),   # checked on the host when de-duplicating
])
def test_upload_rejects_invalid_host_input(n, m, rp, col, flags, msg):
    import paper_2302_03245_amd as pr

    L = pr.lib()
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col if col else [0], np.int32)
    h = ctypes.c_void_p()
    st = L.pr_graph_upload(n, m, rp.ctypes.data, col.ctypes.data, flags, ctypes.byref(h))
    assert st == pr.PR_EINVAL
    assert msg in L.pr_last_error().decode()
    assert h.value is None


def _set_args(graphs):
    rps = [np.asarray(rp, np.int64) for rp, _ in graphs]
    cols = [np.asarray(c if c else [0], np.int32) for _, c in graphs]
    ns = np.array([len(r) - 1 for r in rps], np.int64)
    return (rps, cols, ns, (ctypes.c_void_p * len(rps))(*[r.ctypes.data for r in rps]),
            (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols]))


@pytest.mark.parametrize("graphs,flags,msg", [
    ([([0, 1, 1], [1]), ([0], [])], 0, "n >= 1"),
    ([([0, 1, 1], [1]), ([0, 2, 1], [0, 1])], 0, "non-decreasing"),
    ([([0, 1, 1], [1]), ([1, 1], [0])], 0, "row_ptr[0]"),
    ([([0, 1, 1], [1]), ([0, 1, 1], [2])], 0, "out of [0, n)"),   # an edge into another graph
    ([([0, 1, 1], [1])], 0x2, "unknown upload flag"),
    ([([0, 1, 1], [1])], 0x1, "unknown upload flag"),
    ([([0, 1, 1], [1])], 0x20000, "unknown upload flag"),    # PR_PEEL is not for sets
])
def test_set_upload_rejects_invalid_host_input(graphs, flags, msg):
    import paper_2302_03245_amd as pr

    L = pr.lib()
    rps, cols, ns, rp_ptrs, col_ptrs = _set_args(graphs)
    h = ctypes.c_void_p()
    st = L.pr_set_upload(len(graphs), ns.ctypes.data, rp_ptrs, col_ptrs, flags, ctypes.byref(h))
    assert st == pr.PR_EINVAL
    assert msg in L.pr_last_error().decode()
    assert h.value is None
    st = L.pr_set_upload(0, ns.ctypes.data, rp_ptrs, col_ptrs, 0, ctypes.byref(h))
    assert st == pr.PR_EINVAL and "k must be" in L.pr_last_error().decode()


def test_state_rejects_invalid_host_input():
    import paper_2302_03245_amd as pr

    L = pr.lib()
    h = ctypes.c_void_p()
    assert L.pr_state_create(0, None, ctypes.byref(h)) == pr.PR_EINVAL
    assert "n must be" in L.pr_last_error().decode()
    p = np.array([1.0, -1.0, 2.0])
    assert L.pr_state_create(3, p.ctypes.data, ctypes.byref(h)) == pr.PR_EINVAL
    assert "negative" in L.pr_last_error().decode()
    p = np.zeros(3)
    assert L.pr_state_create(3, p.ctypes.data, ctypes.byref(h)) == pr.PR_EINVAL
    assert "positive sum" in L.pr_last_error().decode()
    assert h.value is None
    out = np.zeros(3)
    assert L.pr_solve_ifp2_warm(None, None, None, out.ctypes.data, None) == pr.PR_EINVAL
    assert L.pr_state_update(None, None, None, None, 0) == pr.PR_EINVAL
    assert L.pr_state_free(None) == pr.PR_OK


def test_set_solve_rejects_null_set():
    import paper_2302_03245_amd as pr

    L = pr.lib()
    out = np.zeros(4)
    assert L.pr_set_solve_ifp2(None, None, None, out.ctypes.data, None) == pr.PR_EINVAL
    assert "graph set is NULL" in L.pr_last_error().decode()
    assert L.pr_set_free(None) == pr.PR_OK


def test_solve_rejects_null_graph_and_bad_options():
    import paper_2302_03245_amd as pr

    L = pr.lib()
    out = np.zeros(4)
    st = L.pr_solve_ifp2(None, None, None, out.ctypes.data, None)
    assert st == pr.PR_EINVAL and "graph is NULL" in L.pr_last_error().decode()
    st = L.pr_ppr(None, None, 0, None, out.ctypes.data, None)
    assert st == pr.PR_EINVAL
    assert L.pr_graph_free(None) == pr.PR_OK


def test_no_cpu_fallback_when_library_missing(monkeypatch):
    import paper_2302_03245_amd as pr

    monkeypatch.setattr(pr, "_lib", None)
    monkeypatch.setattr(pr, "LIB_PATH", LIB + ".missing")
    with pytest.raises(RuntimeError, match="not built"):
        pr.lib()
