"""pr_solve_ifp2_noalloc (the IFP2 solve with its workspace in the library's fixed device
array) against pr_solve_ifp2 and the oracle, through the C ABI: two calls in a row, the
second on a smaller graph (the array keeps the first call's contents), with host and
device outputs, FP64 and FP32 residuals; a solve whose workspace exceeds the array is
rejected with PR_EINVAL and its size."""
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


def test_noalloc_matches_allocating_solve(pr):
    import torch
    big = prgen.random_digraph(70001, 420000, seed=3, dangling_frac=0.15, unref_frac=0.1)
    small = prgen.workload_rmat_small(seed=0)
    for g in (big, small):  # second call: smaller input in the same array
        print(f"noalloc n={g.n} m={g.m}", flush=True)
        ref, _, _ = oracle.power(g, C, tol=1e-13)
        dg = pr.upload(g.row_ptr, g.col)
        for residual, kw, tol in (("fp64", dict(xi=1e-13), 1e-9), ("fp32", dict(l1_tol=1e-6), 1e-6)):
            want, sw = pr.ifp2(dg, c=C, residual=residual, **kw)
            got, sg = pr.ifp2_noalloc(dg, c=C, residual=residual, **kw)
            assert sg["status"] == 0 and sw["status"] == 0
            assert sg["sweeps"] == sw["sweeps"] and sg["vertex_pushes"] == sw["vertex_pushes"]
            assert l1(got, ref) <= tol and l1(got, want) <= 2 * tol
            assert abs(sg["l1_bound"] - sw["l1_bound"]) <= 1e-3 * sw["l1_bound"] + 1e-15
            dev = torch.empty(g.n, dtype=torch.float64, device="cuda")
            _, sd = pr.ifp2_noalloc(dg, c=C, residual=residual, out=dev, **kw)
            assert sd["status"] == 0 and l1(dev.cpu().numpy(), ref) <= tol
        # personalised p (a host vector copied into the array) and a single-source start
        p = prgen.random_p(g.n, seed=3, zero_frac=0.5)
        ref_p, _, _ = oracle.power(g, C, p, tol=1e-13)
        got, sg = pr.ifp2_noalloc(dg, p=p, c=C, xi=1e-13)
        assert sg["status"] == 0 and l1(got, ref_p) <= 1e-9
        dg.free()


def test_noalloc_rejects_oversize(pr):
    n = 12_000_000  # no edges: h, the dangling phase and the host output alone exceed 256 MiB in FP64
    dg = pr.upload(np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32))
    with pytest.raises(pr.PRError) as ei:
        pr.ifp2_noalloc(dg, c=C, xi=1e-12)
    assert ei.value.status == pr.PR_EINVAL and "bytes of workspace" in str(ei.value)
    dg.free()
