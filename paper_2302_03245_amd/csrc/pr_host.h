// pr_host.h -- declarations shared by the host translation units of libpr.so:
// pr_upload.hip (graph upload and plans), pr_solve.hip (the sweep loops of the
// solvers and the autotuner), pr_set_host.hip (graph sets) and pr_host.hip (the
// C ABI).  Error reporting, device buffers and events, solve workspaces and
// option checks live here.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pr.h"
#include "../../include/pr_set.h"
#include "../../include/pr_warm.h"
#include "pr_internal.h"

namespace prk {
namespace host {

// message of the calling thread's last error (pr_last_error)
extern thread_local std::string g_err;

// per-sweep record of the calling thread's last PR_PROFILE solve
struct TraceRec {
    std::vector<int64_t> active, edges;
    std::vector<double> residual, bound;
    std::vector<int32_t> pulled;
};
extern thread_local TraceRec g_trace;

pr_status fail(pr_status st, const std::string &msg);
pr_status hip_fail(hipError_t e, const char *what);

#define HIPCHK(...)                                               \
    do {                                                          \
        hipError_t _e = (__VA_ARGS__);                            \
        if (_e != hipSuccess) return hip_fail(_e, #__VA_ARGS__);  \
    } while (0)

// device buffers freed at scope exit unless released
struct DevBufs {
    std::vector<void *> ptrs;
    ~DevBufs() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t alloc(T **p, size_t count) {
        *p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void **)p, count * sizeof(T));
        if (e == hipSuccess) ptrs.push_back((void *)*p);
        return e;
    }
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t clock_now_ns();
double elapsed_s(hipEvent_t a, hipEvent_t b);

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    explicit EventPair(bool create = true) {
        if (!create) return;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// options (pr_host.hip)
pr_status check_opts(const pr_opts &o, bool power);
pr_status opts_or_default(const pr_opts *o, pr_opts *out);
pr_status enter(const pr_graph *g);

// Solve workspace: one contiguous device allocation (cached on the graph) plus
// a pinned host copy of the control block.
struct Workspace {
    Graph *g = nullptr;
    char *base = nullptr;
    size_t bytes = 0;
    bool cached = false;
    bool borrowed = false;  // caller-provided device memory and host control block: not freed
    Ctl *hctl = nullptr;  // pinned
    hipStream_t stream = nullptr;  // the solve's stream
    ~Workspace() {
        // an error path may leave kernels that use the workspace in flight: wait for them
        // before another solve can take it (a no-op after a solve that finished)
        if (base) (void)hipStreamSynchronize(stream);
        if (borrowed) return;
        if (hctl && !cached) (void)hipHostFree(hctl);
        if (!base) return;
        if (cached) {
            std::lock_guard<std::mutex> lk(g->ws_mu);
            g->ws_busy = false;
        } else {
            (void)hipFree(base);
        }
    }
};


pr_status acquire_ws(Graph &G, size_t bytes, Workspace &ws, hipStream_t s);

// A solve (or a server) holds a use of its graph while it runs; the autotuner, which
// rebuilds the graph's plans, runs only on an unused graph, and solves that start
// while it runs fail with PR_EBUSY.
struct GraphUse {
    Graph *g = nullptr;
    GraphUse() = default;
    GraphUse(const GraphUse &) = delete;
    GraphUse &operator=(const GraphUse &) = delete;
    ~GraphUse() { release(); }
    void release();
};
pr_status use_graph(const Graph &G, GraphUse &u);
struct TuneLock {
    Graph *g = nullptr;
    ~TuneLock();
};
pr_status lock_for_tuning(Graph &G, TuneLock &t);

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count) {
        T *p = (T *)(base + off);
        off += align_up(std::max<size_t>(count, 1) * sizeof(T), 256);
        return p;
    }
};

template <typename T>
size_t carve_size(size_t count) {
    return align_up(std::max<size_t>(count, 1) * sizeof(T), 256);
}

// Validate p (host or device) and place it on the device; returns 1/sum(p).
pr_status prepare_p(const Graph &G, const double *p, const pr_opts &o, double *pdev, double *sumbad,
                    const double **p_used, double *pscale, hipStream_t s);

// Sweep batches: the kernels of sweeps past the stop decision return at once,
// so the host enqueues a batch, reads the control block, and sizes the next
// batch from the observed decay of the certified bound.
int next_batch(int prev_batch, double bound_prev, double bound_now, int swept, double tol, bool l1);

struct SweepTimer {
    bool on = false;
    std::vector<std::unique_ptr<EventPair>> ev;  // per launch
    std::vector<int> sweep_of;                   // sweep index of each launch
    std::vector<int> is_pull;                    // 1 = gather kernel, 0 = scatter kernel
    std::vector<double> bytes;                   // algorithmic bytes of a gather launch
    // events for the next timed launch (taken by the launch itself)
    KernelEvents next(int t, int pull, double b) {
        if (!on) return KernelEvents();
        ev.emplace_back(new EventPair());
        sweep_of.push_back(t);
        is_pull.push_back(pull);
        bytes.push_back(b);
        return KernelEvents{ev.back()->a, ev.back()->b};
    }
};

// partials of one solve: the synchronous sweep's 5 x kRedBlocks, or the ordered
// sweep's 5 x kGroupBlocks per group plus kRedBlocks for the residual sum; a
// group's reserve takes one workgroup per 1024 vertices, up to kGroupBlocks
constexpr size_t kPartDoubles = (size_t)5 * kGroupBlocks * kMaxGroups + kRedBlocks;
static_assert(kPartDoubles >= (size_t)5 * kRedBlocks, "partials");

// state of a warm start (device, original ids): read at the start, written at the end
struct WarmArgs {
    double *pibar;
    double *h;
};

// Device memory a caller provides for a solve's workspace (no allocation in the solve:
// no workspace, pinned control block or timing events are created).
struct ExtWorkspace {
    void *base;
    size_t bytes;
    Ctl *hctl;  // host copy of the control block (any host memory)
};

// ---- graph upload and plans (pr_upload.hip)
pr_status upload_impl(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                      const int32_t *seg_of, pr_graph **out);
// One plan of G (its split-point array owned by G) rebuilt for tiles of kBlock * tile_k items.
hipError_t replan_plan(Graph &G, MPPlan &p, int32_t tile_k, hipStream_t s);
// Every single-vector merge-path plan of the graph rebuilt for tiles of kBlock * tile_k
// items (the batched kernels keep their own plans).
pr_status replan(Graph &G, int32_t tile_k, hipStream_t s);
// The vertex groups of ordered sweeps rebuilt for k groups (k <= 1: none), with their
// whole-row and reached-row gather plans at the graph's current tile size.
pr_status build_groups(Graph &G, int32_t k, hipStream_t s);

// ---- solves (pr_solve.hip)
template <typename T>
pr_status solve_ifp_t(const Graph &G, bool ifp2, const double *p, int32_t source, const pr_opts &o, double *pi,
                      pr_stats *st, const WarmArgs *warm = nullptr, const ExtWorkspace *ext = nullptr);
// Builds and caches on G the stop rule's per-vertex error weights for factor c.
pr_status stop_weights(Graph &G, double c, hipStream_t s);
// Workspace bytes solve_ifp_t takes for these options (the size an ExtWorkspace must have).
template <typename T>
size_t solve_ifp_bytes(const Graph &G, bool ifp2, const double *p, const pr_opts &o, bool warm);
template <typename WT>
pr_status solve_power_t(const Graph &G, const double *p, const pr_opts &o, double *pi, pr_stats *st);
template <typename T, int B>
pr_status solve_ppr_batch_t(const Graph &Gc, const int32_t *srcs, int kb, const pr_opts &o, double *pi_rows,
                            pr_stats *st);
pr_status tune_impl(Graph &G, const pr_opts &o, int32_t reps, pr_tune_report *rep);

}  // namespace host
}  // namespace prk

struct pr_graph_set {
    pr_graph *u = nullptr;                 // the block-diagonal union
    int32_t k = 0;
    std::vector<int64_t> n_g, off;         // vertices per graph; offsets in original ids (k + 1)
    std::vector<int32_t> offN, offD;       // segment offsets in the two regions of the union (k + 1)
    std::vector<int64_t> m_g, mND_g;       // edges, and edges into dangling vertices, per graph
    int32_t *d_offN = nullptr, *d_offD = nullptr;
    uint2 *d_tg_push = nullptr;            // graph range of every tile of the push plan
    std::vector<uint2 *> d_tg_pull;        // ... and of every epoch's gather plan
    // ordered sweeps: every graph's non-dangling vertices split into ngr groups of equal
    // N -> N out-edges (as for one graph); group q of all graphs is a position range
    // [0, glen[q]) cut by d_goff[q] (k + 1) with vertex = position + d_gbase[q][graph]
    int32_t ngr = 1;
    bool prefer_ordered = true;            // set by the autotuner
    std::vector<int32_t> glen;
    std::vector<int32_t *> d_goff, d_gbase;
    std::vector<prk::MPPlan> grp_pull;     // gather plan of each group's in-edges (owned by the union)
    std::vector<uint2 *> d_tg_grp;         // graph range of every tile of those plans
    ~pr_graph_set() {
        if (d_offN) (void)hipFree(d_offN);
        if (d_offD) (void)hipFree(d_offD);
        if (d_tg_push) (void)hipFree(d_tg_push);
        for (uint2 *p : d_tg_pull)
            if (p) (void)hipFree(p);
        for (int32_t *p : d_goff)
            if (p) (void)hipFree(p);
        for (int32_t *p : d_gbase)
            if (p) (void)hipFree(p);
        for (uint2 *p : d_tg_grp)
            if (p) (void)hipFree(p);
        if (u) (void)pr_graph_free(u);
    }
};

struct pr_state {
    int64_t n = 0;
    double c = 0.0;  // fixed by the first solve
    int device = 0;
    double *pibar = nullptr, *h = nullptr;  // device, original ids
    ~pr_state() {
        if (pibar) (void)hipFree(pibar);
        if (h) (void)hipFree(h);
    }
};

namespace prk {
namespace host {

// ---- graph sets (pr_set_host.hip)
pr_status set_upload_impl(int32_t k, const int64_t *n, const int64_t *const *row_ptr, const int32_t *const *col,
                          uint32_t flags, pr_graph_set **out);
template <typename T>
pr_status solve_set_t(const pr_graph_set &S, const double *cg, const pr_opts &o, double *pi, pr_stats *st);
pr_status set_tune_impl(pr_graph_set &S, const double *cg, const pr_opts &o, int32_t reps, pr_tune_report *rep);

}  // namespace host
}  // namespace prk
