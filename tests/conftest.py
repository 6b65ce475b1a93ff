import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size workload (tens of seconds)")


def _ensure_built():
    """Build the CPU-side libraries if nothing is built yet (gcc only, seconds)."""
    import prgen
    import oracle
    if not os.path.exists(os.path.join(ROOT, "prgen", "libprgen.so")):
        from prgen.build import build
        build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        from oracle.build import build as obuild
        obuild()
    return prgen, oracle


_ensure_built()


def l1(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).sum())


def covered(st, got, ref, tol, ref_err=1e-12):
    """L1 distance of a result from the oracle's, checked against the run's gate tol and
    against the run's own reported bound, which must cover the error: l1_verified when the
    run checked its result (PR_VERIFY, a bound for the computed vector in any residual
    precision), else l1_bound (the stop rule's: a certificate with FP64 residuals; with
    FP32 residuals an estimate that leaves out the rounding of the pushes, so FP32 runs
    whose target is near FP32's rounding floor, or whose residuals may all drain to zero,
    must verify or be checked against the gate alone).  ref_err: the reference's own
    error (c / (1 - c) times the oracle's power-method tolerance, or FP64 rounding against
    an exact vector).  Returns the distance."""
    d = l1(got, ref)
    assert d <= tol, (d, tol)
    b = st["l1_verified"] if st.get("l1_verified", 0.0) > 0.0 else st["l1_bound"]
    assert b >= d - ref_err, (st["l1_verified"], st["l1_bound"], d)
    return d


# caps on eps_inf = max |got - ref| for the top-k tie rule, by residual precision
EPS_CAP = {"fp64": 1e-12, "fp32": 1e-9}


def topk_agree(ref, got, k, precision):
    """Top-k ranking check with the tie rule: rank by (value desc, id asc) in both
    vectors; position j may differ only if the two ids' reference values differ by
    at most 2 * eps_inf, where eps_inf = max |got - ref|, and eps_inf itself must not
    exceed the cap of the run's residual precision (1e-12 for FP64, 1e-9 for FP32;
    without the cap a loose result would widen its own tie window).
    Returns (ok, swaps, eps)."""
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    n = ref.size
    k = min(k, n)
    ids = np.arange(n)
    r_order = np.lexsort((ids, -ref))[:k]
    g_order = np.lexsort((ids, -got))[:k]
    eps = float(np.abs(got - ref).max())
    if eps > EPS_CAP[precision]:
        return False, 0, eps
    swaps = 0
    for a, b in zip(r_order, g_order):
        if a == b:
            continue
        swaps += 1
        if abs(ref[a] - ref[b]) > 2 * eps:
            return False, swaps, eps
    return True, swaps, eps


def oracle_many(jobs, workers=None):
    """Run oracle.power over many (graph, c, p, tol) jobs in a thread pool (the oracle is
    a C library called through ctypes, which releases the GIL); returns the vectors in
    job order."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(oracle.power, g, c, p, tol) for (g, c, p, tol) in jobs]
        return [f.result()[0] for f in futs]


@pytest.fixture(scope="session")
def libs():
    return _ensure_built()
