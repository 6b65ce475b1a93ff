"""Benchmark: IFP2 forward-push PageRank vs the power method on one MI355X.

Workload: R-MAT scale 22 (4,194,304 vertices, 16 * 2^22 draws, a/b/c/d =
.57/.19/.19/.05, self-loops and repeats removed), out-edges of a random 15 % of
vertices dropped (dangling), in-edges of a further 10 % redirected
(unreferenced); c = 0.85, uniform p, FP32 residuals with FP64 reserve, stop at a
certified L1 error <= 1e-6.  The graph is resident in HBM before timing; one
step is one complete IFP2 solve (initialisation, sweeps, dangling phase,
normalisation into a device buffer).  The power method is timed the same way.

Prints ONE JSON line (rank 0).  value = normalised GTEPS of IFP2 = m / time to
certified L1 <= 1e-6.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

# The served leg runs one engine per graph, each on its own HIP stream; with HIP's default
# of 4 hardware queues per process, 33 engines share queues and a long kernel of the big
# graph's engine holds up the small graphs' kernels queued behind it.  The process takes
# at least 16 queues, raising a lower setting (HIP reads it once, when it starts; the other
# legs use one or two streams).
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
os.environ["GPU_MAX_HW_QUEUES"] = str(max(_hwq, 16))

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, vendor figure


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha(kernel: str = "pull", kernels_src=None, device_src=None):
    """Hash of the code the counters depend on: the kernel's own text in
    pr_kernels.hip (template line through its closing brace) and the device helpers,
    with comments and blank lines removed (a comment edit keeps the counters valid)."""
    csrc = os.path.join(ROOT, "paper_2302_03245_amd", "csrc")
    src = kernels_src if kernels_src is not None else open(os.path.join(csrc, "pr_kernels.hip")).read()
    dev = device_src if device_src is not None else open(os.path.join(csrc, "pr_device.h")).read()
    start = src.index(f"void k_{kernel}(")
    start = src.rindex("template", 0, start)
    end = src.index("\n}\n", start) + 3

    def code(text):
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.split("\n")]
        return "\n".join(ln for ln in lines if ln.strip())
    body = code(src[start:end]) + "\n" + code(dev)
    return hashlib.sha1(body.encode()).hexdigest()[:12]


def traffic_from_profiles(kernel: str, workload: str, alg_bytes_per_launch: float, tile_items: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source, with the same workgroup tile and on launches of the
    same size (algorithmic bytes per launch within 1 %: one group's gather of an ordered
    sweep, or a synchronous sweep's whole gather); else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_t{tile_items}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha") != kernel_source_sha(kernel) or d.get("tile_items") != tile_items:
        return None
    ref = d.get("algorithmic_bytes_per_launch") or 0.0
    if abs(ref - alg_bytes_per_launch) > 0.01 * alg_bytes_per_launch:
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu():
    """Model name and usable core count of the host running the bench."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(g, c, tol):
    """The serial oracle's IFP2 on the same graph, with the threshold at which an
    empty frontier certifies the same L1 bound (one host core), compiled for this host
    with -O3 -march=native."""
    import tempfile

    import numpy as np

    import oracle
    from oracle.build import build_native
    flags = "-O3 -march=native -ffp-contract=off"
    try:
        d = tempfile.mkdtemp(prefix="oracle_native_")
        oracle.use_library(build_native(os.path.join(d, "liboracle_native.so")))
    except Exception as e:  # keep the portable build if gcc cannot target this host
        log(f"[bench] native oracle build failed ({e}); timing the portable -O2 build")
        flags = "-O2"
    deg = np.diff(g.row_ptr)
    n_nd = int((deg > 0).sum())
    xi = oracle.xi_for_l1(tol, c, g.n, n_nd)
    t0 = time.perf_counter()
    r = oracle.ifp2(g, c, xi=xi)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"one full serial IFP2 solve (oracle, xi={xi:.3e}) on the whole workload graph",
            "seconds": dt, "passes": r["passes"], "build": f"gcc {flags}", "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--workload", default="rmat", choices=["rmat", "dag"],
                    help="rmat: the R-MAT scale-22 workload (the bench line); dag: the layered-DAG workload")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--mode", default=None, choices=[None, "push", "pull"])
    ap.add_argument("--tile-shift", type=int, default=0, help="sweep tile = 256 << s items (s in 2..4; 0 default)")
    ap.add_argument("--groups", type=int, default=0,
                    help="vertex groups of ordered sweeps at upload (0: the library's default)")
    ap.add_argument("--group-all-rows", action="store_true",
                    help="group gathers over every row (to reproduce a tuned schedule with --no-tune)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probes", action="store_true", help="also run the copy / gather / scatter probes")
    ap.add_argument("--ppr", type=int, default=16,
                    help="single-source PPR queries timed one at a time and batched (0 = skip)")
    ap.add_argument("--no-tune", action="store_true", help="skip the per-graph schedule autotuner")
    ap.add_argument("--no-warm", action="store_true", help="skip the dynamic-graph warm-start leg")
    ap.add_argument("--no-peel", action="store_true", help="skip the weak-dangling peeling leg")
    ap.add_argument("--no-ifp1", action="store_true", help="skip the IFP1 leg")
    ap.add_argument("--no-small", action="store_true", help="skip the n = 10,000 FP64 launch-bound leg")
    ap.add_argument("--no-dag", action="store_true", help="skip the layered-DAG leg (IFP2 / IFP1 / power / peeled)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-residual leg on the main graph")
    ap.add_argument("--set-count", type=int, default=256,
                    help="batched solves: independent graphs solved as one set (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="served scenario: seconds of Poisson arrivals (0 = skip)")
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=16, help="served scenario: batch columns per graph (8 or 16)")
    ap.add_argument("--serve-compare", type=int, default=160,
                    help="queries of the served stream also run one at a time and all at once")
    ap.add_argument("--serve-ppr-scale", type=int, default=24,
                    help="R-MAT scale of the resident PPR graph of the served scenario")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2302_03245_amd as pr
    import prgen

    c = 0.85
    t0 = time.perf_counter()
    if args.workload == "rmat":
        log(f"[bench] generating R-MAT scale {args.scale}")
        g = prgen.workload_rmat(scale=args.scale, edge_factor=16, dangling_frac=0.15, unref_frac=0.10, seed=0)
        wl_name = f"R-MAT scale {args.scale}, edge factor 16, 15% dangling, 10% unreferenced, seed 0"
        wl_key = f"rmat{args.scale}"
    else:
        log("[bench] generating the layered DAG (2^23 vertices, 64 layers, 80M Zipf edges + 2% back edges)")
        g = prgen.workload_dag()
        wl_name = "layered DAG: 2^23 vertices in 64 layers, Zipf(2.0) out-degrees capped at 10^4, 80M forward + 2% back edges, seed 0"
        wl_key = "dag23"
    log(f"[bench] n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f}s")
    dg = pr.upload(g.row_ptr, g.col, tile_shift=args.tile_shift, groups=args.groups,
                   group_rows=not args.group_all_rows)
    log(f"[bench] uploaded: {dg.info()}")
    tuning = None
    if not args.no_tune and args.mode is None and args.tile_shift == 0:
        # one-time per graph, like the upload: pick the sweep schedule of global solves
        tuning = pr.tune(dg, c=c, l1_tol=args.tol, residual="fp32", reps=2)
        log(f"[bench] tuned in {tuning['seconds']:.2f}s: chosen {tuning['chosen']}; candidates {tuning['candidates']}")
    info = dg.info()
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")

    def run_ifp2(profile=False):
        return pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, mode=args.mode, profile=profile)

    def run_ifp1(profile=False):
        return pr.ifp1(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, mode=args.mode, profile=profile)

    def run_power(profile=False):
        return pr.power(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, profile=profile)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # HIP events around every sweep kernel of the last timed step only (the roofline
        # figures); the other steps run without them
        stats = [fn(i == args.steps - 1)[1] for i in range(args.steps)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, stats

    log("[bench] IFP2 timed steps")
    t_ifp2, st_ifp2 = timed(run_ifp2)
    log(f"[bench] IFP2 {t_ifp2 * 1e3:.3f} ms/step, sweeps {st_ifp2[-1]['sweeps']}, bound {st_ifp2[-1]['l1_bound']:.3e}")
    t_ifp1, st_ifp1 = None, []
    if not args.no_ifp1:
        log("[bench] IFP1 timed steps")
        t_ifp1, st_ifp1 = timed(run_ifp1)
        log(f"[bench] IFP1 {t_ifp1 * 1e3:.3f} ms/step, sweeps {st_ifp1[-1]['sweeps']}, "
            f"bound {st_ifp1[-1]['l1_bound']:.3e}")
    log("[bench] power method timed steps")
    t_pow, st_pow = timed(run_power)
    log(f"[bench] power {t_pow * 1e3:.3f} ms/step, iterations {st_pow[-1]['sweeps']}")
    assert all(s["status"] == 0 and s["l1_bound"] <= args.tol for s in st_ifp2 + st_ifp1 + st_pow)

    # dominant kernel of the IFP2 step: the scatter (push) or gather (pull) kernel
    prof = st_ifp2[-1:]
    push_s = sum(s["push_seconds"] for s in prof)
    pull_s = sum(s["pull_seconds"] for s in prof)
    kern = "push" if push_s >= pull_s else "pull"
    secs = push_s if kern == "push" else pull_s
    launches = sum(s[f"{kern}_launches"] for s in prof)
    kbytes = sum(s[f"{kern}_bytes"] for s in prof)
    achieved = kbytes / secs / 1e9 if secs > 0 else 0.0
    traffic = traffic_from_profiles(kern, wl_key, kbytes / max(launches, 1), int(info["tile_items"]))
    avg_s = secs / max(launches, 1)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                "traffic_gbs": traffic / avg_s / 1e9 if traffic and avg_s > 0 else None,
                "kernel": f"k_{kern}<float>",
                "launches": launches, "avg_launch_us": secs / max(launches, 1) * 1e6,
                "algorithmic_bytes_per_launch": kbytes / max(launches, 1)}

    last = st_ifp2[-1]
    trace = pr.last_trace()
    log("[bench] IFP2 sweeps: active edges / residual")
    for t in range(len(trace["active"])):
        log(f"  sweep {t:3d} active {trace['active'][t]:9d} edges {trace['edges'][t]:10d} "
            f"residual {trace['residual'][t]:.3e} bound {trace['bound'][t]:.3e} pull {trace['pulled'][t]}")
    res = {
        "metric": "GTEPS + HBM GB/s, IFP2 vs power method at L1<=1e-6; batched/served p50/p99",
        "value": g.m / t_ifp2 / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_ifp2 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl_name,
                   "n": g.n, "m": g.m, "n_dangling": info["n_dangling"], "m_dangling": info["m_dangling"],
                   "n_unreferenced": info["n_unreferenced"], "c": c, "l1_tol": args.tol,
                   "residual": "fp32 residual, fp64 reserve and reductions", "stop": "certified L1"},
        "roofline": roofline,
        "ifp2": {"ms": t_ifp2 * 1e3, "sweeps": last["sweeps"], "pull_sweeps": last["pull_sweeps"],
                 "edges_processed": last["edges_processed"], "edges_traversed": last["edges_traversed"],
                 "gteps_processed": last["edges_processed"] / t_ifp2 / 1e9, "l1_bound": last["l1_bound"],
                 "preprocess_ms": info["seconds_split"] * 1e3},
        "ifp1": None if t_ifp1 is None else {
            "ms": t_ifp1 * 1e3, "sweeps": st_ifp1[-1]["sweeps"], "pull_sweeps": st_ifp1[-1]["pull_sweeps"],
            "edges_processed": st_ifp1[-1]["edges_processed"], "gteps_normalised": g.m / t_ifp1 / 1e9,
            "gteps_processed": st_ifp1[-1]["edges_processed"] / t_ifp1 / 1e9, "l1_bound": st_ifp1[-1]["l1_bound"]},
        "power": {"ms": t_pow * 1e3, "iterations": st_pow[-1]["sweeps"], "gteps_normalised": g.m / t_pow / 1e9,
                  "gteps_processed": st_pow[-1]["edges_processed"] / t_pow / 1e9,
                  "l1_bound": st_pow[-1]["l1_bound"]},
        "ifp2_over_power": t_pow / t_ifp2,
        "upload_s": info["seconds_upload"],
        "tuning": tuning,
        "schedule": {"tile_items": info["tile_items"], "ordered_sweeps": bool(info["ordered"]),
                     "groups": info["groups"]},
        "depth_epochs": info["epochs"], "max_depth": info["max_depth"],
    }
    # one verified solve of the timed configuration: the a-posteriori bound of the result
    # (the solve sweeps on, and says how far, when the check finds the stop rule's result short)
    _, stv = pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, mode=args.mode, verify=True)
    res["ifp2"]["l1_verified"] = stv["l1_verified"]
    res["ifp2"]["verified_sweeps"] = stv["sweeps"]
    res["ifp2"]["verified_status"] = stv["status"]
    res["ifp2"]["launches"] = last["launches"]
    _, stv = pr.power(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, verify=True)
    res["power"]["l1_verified"] = stv["l1_verified"]
    log(f"[bench] verified bounds: IFP2 {res['ifp2']['l1_verified']:.3e}, power {res['power']['l1_verified']:.3e}")
    if not args.no_fp64 and args.mode is None:
        res["fp64"] = run_fp64(pr, dg, g, c, args, out)
    if not args.no_peel and args.mode is None:
        res["peeled"] = run_peel(pr, g, c, args, t_ifp2, last)
    if args.ppr > 0:
        res["ppr"] = run_ppr(pr, dg, g, c, args)
    if not args.no_warm:
        res["warm_start"] = run_warm(pr, prgen, dg, g, c, args)
    if args.set_count > 0:
        res["batched_graphs"] = run_set(pr, prgen, args)
    if args.serve_seconds > 0:
        res["served"] = run_serve(pr, prgen, c, args)
    if args.probes:
        res["probes"] = run_probes(pr, torch, g)
    if not args.no_small:
        res["small_fp64"] = run_small(pr, prgen, args)
    if not args.no_dag and args.workload == "rmat":
        dg.free()
        res["dag"] = run_dag(pr, prgen, c, args)
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (serial oracle IFP2)")
        res["cpu_baseline"] = cpu_baseline(g, c, args.tol)
    print(json.dumps(res), flush=True)


def _timed(fn, steps, warmup):
    """Mean wall time of `steps` calls after `warmup` (device synchronised around), and
    the stats of the last call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, st


def run_fp64(pr, dg, g, c, args, out):
    """The main graph with FP64 residuals at L1 <= 1e-9 (the paper computes in FP64), IFP2
    against the FP64 power method at the same certified accuracy."""
    tol = 1e-9
    t2, s2 = _timed(lambda: pr.ifp2(dg, c=c, l1_tol=tol, out=out), args.steps, args.warmup)
    tp, sp = _timed(lambda: pr.power(dg, c=c, l1_tol=tol, out=out), args.steps, args.warmup)
    _, v2 = pr.ifp2(dg, c=c, l1_tol=tol, out=out, verify=True)
    assert s2["status"] == 0 and s2["l1_bound"] <= tol and sp["status"] == 0
    res = {"l1_tol": tol, "ifp2_ms": t2 * 1e3, "ifp2_sweeps": s2["sweeps"], "ifp2_gteps": g.m / t2 / 1e9,
           "ifp2_l1_bound": s2["l1_bound"], "ifp2_l1_verified": v2["l1_verified"],
           "power_ms": tp * 1e3, "power_iterations": sp["sweeps"], "power_gteps": g.m / tp / 1e9,
           "ifp2_over_power": tp / t2}
    log(f"[bench] fp64: {res}")
    return res


def run_small(pr, prgen, args):
    """The correctness-sized workload: R-MAT n = 10,000, 100,000 distinct edges drawn, 10 %
    forced dangling, c = 0.85, uniform p, FP64 residuals, xi = 1e-12 (Algorithms 2 and 3's
    threshold rule), against the FP64 power method run to the bound IFP2 certified.
    Launch-bound: every array is L2-resident."""
    c = 0.85
    g = prgen.workload_rmat_small(seed=0)
    dg = pr.upload(g.row_ptr, g.col)
    steps = max(args.steps, 20)
    t2, s2 = _timed(lambda: pr.ifp2(dg, c=c, xi=1e-12), steps, args.warmup)
    t1, s1 = _timed(lambda: pr.ifp1(dg, c=c, xi=1e-12), steps, args.warmup)
    tol = s2["l1_bound"]
    tp, sp = _timed(lambda: pr.power(dg, c=c, l1_tol=tol), steps, args.warmup)
    _, v2 = pr.ifp2(dg, c=c, xi=1e-12, verify=True)
    assert s2["status"] == 0 and sp["status"] == 0
    res = {"workload": "R-MAT n=10,000, 100,000 distinct edges drawn, 10% forced dangling, seed 0",
           "n": g.n, "m": g.m, "xi": 1e-12,
           "ifp2_ms": t2 * 1e3, "ifp2_sweeps": s2["sweeps"], "ifp2_launches": s2["launches"],
           "ifp2_us_per_launch": t2 * 1e6 / max(1, s2["launches"]), "ifp2_device_ms": s2["seconds_solve"] * 1e3,
           "ifp2_l1_bound": s2["l1_bound"], "ifp2_l1_verified": v2["l1_verified"],
           "ifp1_ms": t1 * 1e3, "ifp1_sweeps": s1["sweeps"], "ifp1_launches": s1["launches"],
           "power_ms": tp * 1e3, "power_iterations": sp["sweeps"], "power_launches": sp["launches"],
           "power_l1_tol": tol, "ifp2_over_power": tp / t2}
    log(f"[bench] small FP64: {res}")
    dg.free()
    return res


def run_dag(pr, prgen, c, args):
    """The layered-DAG workload (2^23 vertices in 64 layers, Zipf(2.0) out-degrees capped at
    10^4 scaled to 80M forward edges, 2 % back edges): IFP2, IFP1 and the power method with
    FP32 residuals at certified L1 <= tol, and IFP2 on the graph uploaded with its weakly
    dangling vertices peeled; each tuned once like the main graph."""
    import torch
    t0 = time.perf_counter()
    g = prgen.workload_dag()
    log(f"[bench] dag: n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f}s")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    dg = pr.upload(g.row_ptr, g.col)
    if not args.no_tune:
        pr.tune(dg, c=c, l1_tol=args.tol, residual="fp32", reps=2)
    info = dg.info()
    t2, s2 = _timed(lambda: pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=out), args.steps, args.warmup)
    t1, s1 = _timed(lambda: pr.ifp1(dg, c=c, l1_tol=args.tol, residual="fp32", out=out), args.steps, args.warmup)
    tp, sp = _timed(lambda: pr.power(dg, c=c, l1_tol=args.tol, residual="fp32", out=out), args.steps, args.warmup)
    t0 = time.perf_counter()
    _, v2 = pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=out, verify=True)
    torch.cuda.synchronize()
    tv = time.perf_counter() - t0
    dg.free()
    dp = pr.upload(g.row_ptr, g.col, peel=True)
    if not args.no_tune:
        pr.tune(dp, c=c, l1_tol=args.tol, residual="fp32", reps=2)
    pinfo = dp.info()
    tq, sq = _timed(lambda: pr.ifp2(dp, c=c, l1_tol=args.tol, residual="fp32", out=out), args.steps, args.warmup)
    dp.free()
    for st in (s2, s1, sp, sq):
        assert st["status"] == 0 and st["l1_bound"] <= args.tol
    res = {"workload": "layered DAG: 2^23 vertices in 64 layers, Zipf(2.0) out-degrees capped at 10^4, "
                       "80M forward + 2% back edges, seed 0",
           "n": g.n, "m": g.m, "lambda": g.meta["lambda"],
           "ifp2_ms": t2 * 1e3, "ifp2_sweeps": s2["sweeps"], "ifp2_gteps": g.m / t2 / 1e9,
           "ifp2_l1_bound": s2["l1_bound"], "ifp2_l1_verified": v2["l1_verified"],
           "ifp2_verified_sweeps": v2["sweeps"], "ifp2_verified_status": v2["status"],
           "ifp2_verified_ms_incl_checks": tv * 1e3,
           "ifp1_ms": t1 * 1e3, "ifp1_sweeps": s1["sweeps"], "ifp1_gteps": g.m / t1 / 1e9,
           "power_ms": tp * 1e3, "power_iterations": sp["sweeps"], "power_gteps": g.m / tp / 1e9,
           "peeled_ms": tq * 1e3, "peeled_sweeps": sq["sweeps"], "peeled_gteps": g.m / tq / 1e9,
           "n_peeled": pinfo["n_peeled"], "peel_levels": pinfo["peel_levels"],
           "ifp2_over_power": tp / t2, "peeled_over_power": tp / tq,
           "schedule": {"tile_items": info["tile_items"], "ordered_sweeps": bool(info["ordered"]),
                        "groups": info["groups"]}}
    log(f"[bench] dag: {res}")
    return res


def run_peel(pr, g, c, args, t_plain, st_plain):
    """IFP2 on the same graph uploaded with its weakly dangling vertices peeled (PR_PEEL:
    phase 1 sweeps the core only, phase 2 gathers the peeled levels from the highest
    down); same options, tuning and step count as the main IFP2 line."""
    import torch
    t0 = time.perf_counter()
    dp = pr.upload(g.row_ptr, g.col, tile_shift=args.tile_shift, peel=True)
    t_up = time.perf_counter() - t0
    if not args.no_tune and args.tile_shift == 0:
        pr.tune(dp, c=c, l1_tol=args.tol, residual="fp32", reps=2)
    info = dp.info()
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        pr.ifp2(dp, c=c, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [pr.ifp2(dp, c=c, l1_tol=args.tol, residual="fp32", out=out)[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    assert all(s["status"] == 0 and s["l1_bound"] <= args.tol for s in sts)
    st = sts[-1]
    res = {"ms": t * 1e3, "gteps": g.m / t / 1e9, "speedup_vs_unpeeled": t_plain / t,
           "n_peeled": info["n_peeled"], "levels": info["peel_levels"],
           "edges_processed": st["edges_processed"], "edges_processed_unpeeled": st_plain["edges_processed"],
           "sweeps": st["sweeps"], "l1_bound": st["l1_bound"], "upload_s": t_up,
           "ordered_sweeps": bool(info["ordered"]), "tile_items": info["tile_items"]}
    log(f"[bench] peeled: {res}")
    dp.free()
    return res


def run_ppr(pr, dg, g, c, args):
    """Aggregate throughput of single-source PPR (IFP2, FP32 residuals, certified L1 <= tol):
    the same queries one call per source, and in one call (batched sixteen per launch)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(7)
    deg = np.diff(g.row_ptr)
    srcs = rng.choice(np.where(deg > 0)[0], args.ppr, replace=False).astype(np.int32)
    out = torch.empty((len(srcs), g.n), dtype=torch.float64, device="cuda")  # results stay in HBM
    pr.ppr(dg, srcs[:2], c=c, l1_tol=args.tol, residual="fp32", out=out[:2])  # warm-up of both paths
    pr.ppr(dg, srcs[:1], c=c, l1_tol=args.tol, residual="fp32", out=out[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = [pr.ppr(dg, srcs[i:i + 1], c=c, l1_tol=args.tol, residual="fp32", out=out[i:i + 1])[1][0]
              for i in range(len(srcs))]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, batched = pr.ppr(dg, srcs, c=c, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    assert all(s["status"] == 0 and s["l1_bound"] <= args.tol for s in single + batched)
    k = len(srcs)
    log(f"[bench] PPR x{k}: one at a time {t_single * 1e3:.1f} ms, batched {t_batch * 1e3:.1f} ms")
    return {"queries": k, "one_at_a_time_ms": t_single * 1e3, "batched_ms": t_batch * 1e3,
            "one_at_a_time_gteps": k * g.m / t_single / 1e9, "batched_gteps": k * g.m / t_batch / 1e9,
            "speedup": t_single / t_batch, "batch_width": 16,
            "mean_sweeps_single": float(np.mean([s["sweeps"] for s in single])),
            "mean_sweeps_batched": float(np.mean([s["sweeps"] for s in batched])),
            # the batch's sweeps that gathered, and the edges its sweeps read (gathers: every
            # live in-edge; scatters: the active edges; plus the dangling phase's in-edges)
            "batched_gather_sweeps": int(batched[0]["pull_sweeps"]),
            "batched_edges_traversed": int(batched[0]["edges_traversed"])}


def run_warm(pr, prgen, dg, g, c, args):
    """Dynamic graph: after a solve, the out-edge lists of a random 0.1 % of the
    non-dangling vertices are replaced (random targets, the same number of edges); the
    state is carried to the new graph (pr_state_update over the changed sources) and
    IFP2 resumes from it, against a cold solve of the changed graph; FP32 residuals,
    certified L1 <= tol."""
    import numpy as np
    import torch
    rng = np.random.default_rng(17)
    deg = np.diff(g.row_ptr)
    nz = np.flatnonzero(deg > 0)
    changed = np.sort(rng.choice(nz, max(1, len(nz) // 1000), replace=False)).astype(np.int32)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    keep = ~np.isin(src, changed)
    new_dst = rng.integers(0, g.n, int(deg[changed].sum()))
    new_src = np.repeat(changed.astype(np.int64), deg[changed])
    g2 = prgen.from_edges(g.n, np.concatenate([src[keep], new_src]), np.concatenate([g.col[keep], new_dst]))
    d2 = pr.upload(g2.row_ptr, g2.col)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = pr.State(g.n)
    pr.ifp2_warm(dg, st, c=c, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.update(dg, d2, changed)
    t_upd = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, sw = pr.ifp2_warm(d2, st, c=c, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    def cold(jacobi):
        pr.ifp2(d2, c=c, l1_tol=args.tol, residual="fp32", out=out, jacobi=jacobi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st_c = pr.ifp2(d2, c=c, l1_tol=args.tol, residual="fp32", out=out, jacobi=jacobi)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st_c
    # the changed graph solved from scratch with its default schedule, and with synchronous sweeps
    t_cold, sc = cold(False)
    t_cold_sync, sc_sync = cold(True)
    res = {"changed_sources": int(len(changed)), "changed_edges": int(deg[changed].sum()),
           "update_ms": t_upd * 1e3, "warm_ms": t_warm * 1e3, "cold_ms": t_cold * 1e3,
           "cold_synchronous_ms": t_cold_sync * 1e3, "cold_synchronous_sweeps": sc_sync["sweeps"],
           "warm_sweeps": sw["sweeps"], "cold_sweeps": sc["sweeps"],
           "warm_edges_processed": sw["edges_processed"], "cold_edges_processed": sc["edges_processed"],
           "warm_l1_bound": sw["l1_bound"], "cold_l1_bound": sc["l1_bound"],
           "speedup_incl_update": t_cold / (t_warm + t_upd)}
    log(f"[bench] warm start: {res}")
    st.free()
    d2.free()
    return res


def run_set(pr, prgen, args):
    """Batched solves: independent R-MAT graphs (n log-uniform in [1k, 500k], average
    degree uniform in [4, 32], 5-20 % dangling, c drawn from {0.85, 0.9} per graph)
    solved as one graph set, against the same graphs solved one at a time; IFP2 with
    FP32 residuals, certified L1 <= tol per graph, results in HBM."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    graphs, cs = prgen.workload_batch(count=args.set_count, seed=0)
    n_tot, m_tot = sum(g.n for g in graphs), sum(g.m for g in graphs)
    log(f"[bench] set: {len(graphs)} graphs, n {n_tot}, m {m_tot}, generated in {time.perf_counter() - t0:.1f}s")
    gs = pr.upload_set([(g.row_ptr, g.col) for g in graphs])
    tuning = None
    if not args.no_tune:
        # one-time per set, like the upload: tile size and ordered / synchronous sweeps
        tuning = pr.set_tune(gs, c=cs, l1_tol=args.tol, residual="fp32", reps=2)
        log(f"[bench] set tuned in {tuning['seconds']:.2f}s: chosen {tuning['chosen']}")
    info = gs.info()
    out = torch.empty(gs.n, dtype=torch.float64, device="cuda")
    pr.set_ifp2(gs, c=cs, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        _, sts = pr.set_ifp2(gs, c=cs, l1_tol=args.tol, residual="fp32", out=out)
    torch.cuda.synchronize()
    t_set = (time.perf_counter() - t0) / reps
    ok_set = all(st["l1_bound"] <= args.tol and st["status"] == 0 for st in sts)
    sums = torch.stack([x.sum() for x in gs.split(out)]).cpu().numpy()
    # one at a time: each graph resident on its own (tuned on its own too), solved back to back
    dgs = [pr.upload(g.row_ptr, g.col) for g in graphs]
    if not args.no_tune:
        for dg, c in zip(dgs, cs):
            pr.tune(dg, c=c, l1_tol=args.tol, residual="fp32", reps=1)
    outs = gs.split(out)
    for dg, c, o in zip(dgs[:4], cs, outs):
        pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok_one = True
    for dg, c, o in zip(dgs, cs, outs):
        _, st = pr.ifp2(dg, c=c, l1_tol=args.tol, residual="fp32", out=o)
        ok_one = ok_one and st["l1_bound"] <= args.tol
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    for dg in dgs:
        dg.free()
    res = {"graphs": len(graphs), "n": n_tot, "m": m_tot, "set_ms": t_set * 1e3, "one_at_a_time_ms": t_one * 1e3,
           "gteps_set": m_tot / t_set / 1e9, "gteps_one_at_a_time": m_tot / t_one / 1e9,
           "set_over_one_at_a_time": t_one / t_set, "all_certified": bool(ok_set and ok_one),
           "max_sum_error": float(np.abs(sums - 1.0).max()),
           "sweeps_max": max(st["sweeps"] for st in sts), "sweeps_min": min(st["sweeps"] for st in sts),
           "upload_s": info["seconds_upload"], "device_bytes": info["device_bytes"],
           "schedule": {"groups": info["groups"], "ordered_sweeps": bool(info["ordered"]),
                        "tile_items": info["tile_items"]},
           "tuning": tuning}
    log(f"[bench] set: {res}")
    gs.free()
    return res


def run_serve(pr, prgen, c, args):
    """Served queries: Poisson arrivals at --serve-qps for --serve-seconds; 30 % are
    single-source PPR (uniformly random source) on a resident R-MAT graph of scale
    --serve-ppr-scale (2**28 draws at scale 24), 70 % global PageRank on one of 32
    resident R-MAT graphs (n log-uniform in [10k, 4M], average degree 16, 15 %
    dangling), picked uniformly.  IFP2 with FP32 residuals, certified L1 <= tol per
    query; one server (continuous batching, 16 slots per graph); results stay in HBM.

    Beside the open-loop run, the first --serve-compare queries of the same stream are
    solved one at a time (pr_ppr / pr_solve_ifp2, back to back) and, separately, all
    submitted to the server at once: aggregate GTEPS of both at equal accuracy."""
    import threading

    import numpy as np
    import torch
    log(f"[bench] serve: generating the PPR graph (scale {args.serve_ppr_scale}) and the 32-graph pool")
    t0 = time.perf_counter()
    gp = prgen.workload_rmat(scale=args.serve_ppr_scale, edge_factor=16, dangling_frac=0.15, unref_frac=0.10, seed=1)
    pool = prgen.workload_serve_pool(count=32, seed=0)
    graphs = [gp] + pool
    log(f"[bench] serve: graphs ready in {time.perf_counter() - t0:.1f}s (PPR graph n={gp.n} m={gp.m}; pool "
        f"n {sum(x.n for x in pool)} m {sum(x.m for x in pool)})")
    dgs = [pr.upload(x.row_ptr, x.col) for x in graphs]
    rng = np.random.default_rng(11)
    n_q = int(args.serve_qps * args.serve_seconds)
    gaps = rng.exponential(1.0 / args.serve_qps, n_q)
    is_ppr = rng.random(n_q) < 0.30
    pool_pick = rng.integers(1, len(graphs), n_q)
    srcs = rng.integers(0, gp.n, n_q)
    queries = [(0, int(srcs[q])) if is_ppr[q] else (int(pool_pick[q]), -1) for q in range(n_q)]
    free = [[torch.empty(x.n, dtype=torch.float64, device="cuda") for _ in range(24 if i == 0 else 8)]
            for i, x in enumerate(graphs)]
    big = 1 + int(np.argmax([x.n for x in pool]))

    def make_server():
        srv = pr.Server(c=c, l1_tol=args.tol, residual="fp32", slots=args.serve_slots, sweeps_per_round=4)
        gids = [srv.add_graph(d) for d in dgs]
        for gi in range(len(graphs)):  # one query per graph first: workspaces and plans
            buf = free[gi][0]
            srv.wait(srv.submit(gids[gi], -1, buf), timeout=300.0)
        return srv, gids

    def serve(qs, gaps_s):
        """Submit qs at the given inter-arrival gaps (None: all at once); returns
        per-query (graph index, stats) in completion order and the span."""
        srv, gids = make_server()
        lock = threading.Condition()
        pending, done = [], []

        def collector():
            while True:
                with lock:
                    while not pending:
                        lock.wait()
                    item = pending.pop(0)
                if item is None:
                    return
                rid, gi, buf = item
                st = srv.wait(rid, timeout=300.0)
                with lock:
                    done.append((gi, st))
                    free[gi].append(buf)
                    lock.notify_all()

        th = threading.Thread(target=collector)
        th.start()
        t_start = time.perf_counter()
        t_next = t_start
        for q, (gi, src) in enumerate(qs):
            if gaps_s is not None:
                t_next += gaps_s[q]
                delay = t_next - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            with lock:
                while not free[gi]:
                    lock.wait()
                buf = free[gi].pop()
            rid = srv.submit(gids[gi], src, buf)
            with lock:
                pending.append((rid, gi, buf))
                lock.notify_all()
        with lock:
            pending.append(None)
            lock.notify_all()
        th.join()
        span = time.perf_counter() - t_start
        mem = srv.stats()
        foot = {"ppr_graph": {w: srv.footprint(gids[0], w) for w in (1, 8, 16)},
                "largest_pool_graph": {w: srv.footprint(gids[big], w) for w in (1, 8, 16)}}
        srv.close()
        memory = {"budget_gb": mem["budget"] / 1e9, "graphs_gb": mem["graph_bytes"] / 1e9,
                  "peak_gb": mem["peak_bytes"] / 1e9, "memory_waits": mem["memory_waits"],
                  "narrowed_runs": mem["narrowed_runs"], "rejected": mem["rejected"],
                  "workspace_bytes_by_width": foot}
        return done, span, memory

    def summary(done, span):
        ok = all(st["status"] == 0 and st["l1_bound"] <= args.tol for _, st in done)
        lat = np.array([st["seconds_solve"] for _, st in done]) * 1e3
        kind = np.array([gi == 0 for gi, _ in done])
        edges = sum(graphs[gi].m for gi, _ in done)
        out = {"completed": len(done), "all_certified": ok, "seconds": span, "qps": len(done) / span,
               "gteps_aggregate": edges / span / 1e9,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
        for name, sel in (("ppr", kind), ("pagerank", ~kind)):
            if sel.any():
                out[name] = {"count": int(sel.sum()), "p50_ms": float(np.percentile(lat[sel], 50)),
                             "p99_ms": float(np.percentile(lat[sel], 99))}
        return out

    done, span, memory = serve(queries, gaps)
    open_loop = summary(done, span)
    open_loop.update({"qps_target": args.serve_qps, "queries": n_q, "memory": memory})
    log(f"[bench] served open loop: {open_loop}")

    k = min(args.serve_compare, n_q)
    done, span, _ = serve(queries[:k], None)
    saturated = summary(done, span)
    log(f"[bench] served, {k} queries submitted at once: {saturated}")

    # the same queries one at a time, back to back, same accuracy
    for gi in range(len(graphs)):
        pr.ifp2(dgs[gi], c=c, l1_tol=args.tol, residual="fp32", out=free[gi][0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges, ok = 0, True
    for gi, src in queries[:k]:
        if src >= 0:
            _, sts = pr.ppr(dgs[gi], [src], c=c, l1_tol=args.tol, residual="fp32", out=free[gi][0].view(1, -1))
            st = sts[0]
        else:
            _, st = pr.ifp2(dgs[gi], c=c, l1_tol=args.tol, residual="fp32", out=free[gi][0])
        ok = ok and st["l1_bound"] <= args.tol
        edges += graphs[gi].m
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    one = {"queries": k, "seconds": t_one, "gteps_aggregate": edges / t_one / 1e9, "all_certified": ok}
    log(f"[bench] the same {k} queries one at a time: {one}")
    return {"open_loop": open_loop, "saturated": saturated, "one_at_a_time": one,
            "served_over_one_at_a_time": saturated["gteps_aggregate"] / one["gteps_aggregate"],
            "ppr_graph": {"n": gp.n, "m": gp.m},
            "pool": {"graphs": len(pool), "n": sum(x.n for x in pool), "m": sum(x.m for x in pool)},
            "ppr_share": float(is_ppr.mean()), "slots_per_graph": args.serve_slots,
            "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])}


def run_probes(pr, torch, g):
    import ctypes

    import numpy as np
    L = pr.lib()
    out = {}
    sec = ctypes.c_double()
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    s = torch.cuda.current_stream().cuda_stream
    assert L.pr_probe_copy(a.data_ptr(), b.data_ptr(), nbytes, 10, s, ctypes.byref(sec)) == 0
    out["copy_GBs"] = 2 * nbytes / sec.value / 1e9
    del a, b
    n = g.n
    m = g.m
    idx = torch.tensor(g.col, device="cuda")
    w = torch.ones(n, dtype=torch.float32, device="cuda")
    olen = L.pr_probe_gather_out_len(m)
    o = torch.empty(olen, dtype=torch.float32, device="cuda")
    assert L.pr_probe_gather(w.data_ptr(), idx.data_ptr(), m, o.data_ptr(), olen, 10, s, ctypes.byref(sec)) == 0
    out["gather_rmat_Gidx_s"] = m / sec.value / 1e9
    assert L.pr_probe_scatter(w.data_ptr(), idx.data_ptr(), m, 1.0, 10, s, ctypes.byref(sec)) == 0
    out["scatter_rmat_Gatomics_s"] = m / sec.value / 1e9
    rnd = torch.randint(0, n, (m,), dtype=torch.int32, device="cuda")
    assert L.pr_probe_gather(w.data_ptr(), rnd.data_ptr(), m, o.data_ptr(), olen, 10, s, ctypes.byref(sec)) == 0
    out["gather_uniform_Gidx_s"] = m / sec.value / 1e9
    assert L.pr_probe_scatter(w.data_ptr(), rnd.data_ptr(), m, 1.0, 10, s, ctypes.byref(sec)) == 0
    out["scatter_uniform_Gatomics_s"] = m / sec.value / 1e9
    seq = torch.arange(m, dtype=torch.int32, device="cuda") % n
    assert L.pr_probe_scatter(w.data_ptr(), seq.data_ptr(), m, 1.0, 10, s, ctypes.byref(sec)) == 0
    out["scatter_sequential_Gatomics_s"] = m / sec.value / 1e9
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
