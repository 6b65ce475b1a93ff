// pr_host.hip -- the C ABI of libpr.so (include/pr.h, pr_set.h, pr_warm.h) and the
// host helpers the other host translation units share (errors, options).
#include "pr_host.h"

namespace prk {
namespace host {

thread_local std::string g_err;
thread_local TraceRec g_trace;
// testing hook of pr_ppr: fail on reaching this batch (0: off)
thread_local int32_t t_fail_ppr_batch = 0;

pr_status fail(pr_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

pr_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

int64_t clock_now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

double elapsed_s(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

pr_status check_opts(const pr_opts &o, bool power) {
    if (!(o.c > 0.0 && o.c < 1.0)) return fail(PR_EINVAL, "c must be in (0, 1)");
    if (o.stop != PR_STOP_XI && o.stop != PR_STOP_L1) return fail(PR_EINVAL, "unknown stop rule");
    if (o.residual != PR_RES_FP64 && o.residual != PR_RES_FP32) return fail(PR_EINVAL, "unknown residual type");
    if (o.max_sweeps < 0) return fail(PR_EINVAL, "max_sweeps < 0");
    const uint32_t known =
        PR_P_DEVICE | PR_OUT_DEVICE | PR_IFP2_LITERAL | PR_FORCE_PUSH | PR_FORCE_PULL | PR_PROFILE | PR_JACOBI |
        PR_VERIFY | PR_FORCE_LIST;
    if (o.flags & ~known) return fail(PR_EINVAL, "unknown option flag");
    const uint32_t modes = o.flags & (PR_FORCE_PUSH | PR_FORCE_PULL | PR_FORCE_LIST);
    if (modes & (modes - 1)) return fail(PR_EINVAL, "at most one of PR_FORCE_PUSH, PR_FORCE_PULL, PR_FORCE_LIST");
    if (power || o.stop == PR_STOP_L1) {
        if (!(o.l1_tol > 0.0) || !isfinite(o.l1_tol)) return fail(PR_EINVAL, "l1_tol must be > 0 and finite");
    }
    if (!power && o.stop == PR_STOP_XI) {
        if (!(o.xi > 0.0) || !isfinite(o.xi)) return fail(PR_EINVAL, "xi must be > 0 and finite");
    }
    return PR_OK;
}

pr_status opts_or_default(const pr_opts *o, pr_opts *out) {
    if (o) *out = *o;
    else pr_opts_default(out);
    return PR_OK;
}

pr_status enter(const pr_graph *g) {
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    HIPCHK(hipSetDevice(g->g.device));
    return PR_OK;
}

void GraphUse::release() {
    if (!g) return;
    std::lock_guard<std::mutex> lk(g->ws_mu);
    --g->users;
    g = nullptr;
}

pr_status use_graph(const Graph &Gc, GraphUse &u) {
    Graph &G = const_cast<Graph &>(Gc);
    std::lock_guard<std::mutex> lk(G.ws_mu);
    if (G.tuning) return fail(PR_EBUSY, "the graph is being tuned (pr_graph_tune / pr_set_tune)");
    ++G.users;
    u.g = &G;
    return PR_OK;
}

TuneLock::~TuneLock() {
    if (!g) return;
    std::lock_guard<std::mutex> lk(g->ws_mu);
    g->tuning = false;
}

pr_status lock_for_tuning(Graph &G, TuneLock &t) {
    std::lock_guard<std::mutex> lk(G.ws_mu);
    if (G.users > 0) return fail(PR_EBUSY, "solves or a server are using the graph");
    if (G.tuning) return fail(PR_EBUSY, "the graph is already being tuned");
    G.tuning = true;
    t.g = &G;
    return PR_OK;
}

}  // namespace host

pr_status set_error(pr_status st, const std::string &msg) { return host::fail(st, msg); }
void clear_error() { host::g_err.clear(); }

}  // namespace prk

using namespace prk;
using namespace prk::host;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void pr_opts_default(pr_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->c = 0.85;
    o->xi = 1e-12;
    o->l1_tol = 1e-6;
    o->stop = PR_STOP_XI;
    o->residual = PR_RES_FP64;
}

const char *pr_last_error(void) { return g_err.c_str(); }

int32_t pr_last_trace(int32_t cap, int64_t *active, int64_t *edges, double *residual, double *bound,
                      int32_t *pulled) {
    const int32_t n = (int32_t)g_trace.active.size();
    const int32_t k = std::min(n, std::max<int32_t>(cap, 0));
    for (int32_t i = 0; i < k; ++i) {
        if (active) active[i] = g_trace.active[i];
        if (edges) edges[i] = g_trace.edges[i];
        if (residual) residual[i] = g_trace.residual[i];
        if (bound) bound[i] = g_trace.bound[i];
        if (pulled) pulled[i] = g_trace.pulled[i];
    }
    return n;
}

pr_status pr_graph_upload(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                          pr_graph **out) {
    g_err.clear();
    try {
        return upload_impl(n, m, row_ptr, col, flags, nullptr, out);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_graph_free(pr_graph *g) {
    g_err.clear();
    if (!g) return PR_OK;
    (void)hipSetDevice(g->g.device);
    if (g->g.stream) (void)hipStreamSynchronize(g->g.stream);
    for (void *p : g->g.allocs) (void)hipFree(p);
    for (void *p : g->g.grp_allocs) (void)hipFree(p);
    if (g->g.ws_mem) (void)hipFree(g->g.ws_mem);
    if (g->g.ws_hctl) (void)hipHostFree(g->g.ws_hctl);
    if (g->g.stream) (void)hipStreamDestroy(g->g.stream);
    delete g;
    return PR_OK;
}

pr_status pr_graph_info(const pr_graph *g, pr_graph_info_t *out) {
    g_err.clear();
    if (!g || !out) return fail(PR_EINVAL, "NULL argument");
    const Graph &G = g->g;
    out->n = G.n;
    out->m = G.m;
    out->n_dangling = G.nD - G.nP;
    out->m_dangling = G.mND;
    out->n_unreferenced = G.n_unref;
    out->device_bytes = G.device_bytes;
    out->seconds_upload = G.seconds_upload;
    out->seconds_split = G.seconds_split;
    out->max_depth = G.max_depth;
    out->epochs = (int64_t)G.epochs.size();
    out->groups = G.grp.size() > 1 ? (int64_t)G.grp.size() - 1 : 1;
    out->tile_items = (int64_t)kBlock * G.tile_k;
    out->ordered = G.grp.size() > 2 && !G.grp_pull.empty() && G.prefer_ordered ? 1 : 0;
    out->n_peeled = G.nP;
    out->peel_levels = G.nP > 0 ? (int64_t)G.lvl_pull.size() - 1 : 0;
    return PR_OK;
}

static pr_status solve_common(const pr_graph *g, int method, const double *p, const pr_opts *o, double *pi,
                              pr_stats *st) {
    g_err.clear();
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    if (!pi) return fail(PR_EINVAL, "pi is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    pr_status ps = check_opts(op, method == 3);
    if (ps != PR_OK) return ps;
    ps = enter(g);
    if (ps != PR_OK) return ps;
    if (method == 1 && g->g.nP > 0)
        return fail(PR_EINVAL, "a graph uploaded with PR_PEEL serves IFP2 and power solves, not IFP1");
    GraphUse use;
    ps = use_graph(g->g, use);
    if (ps != PR_OK) return ps;
    try {
        const Graph &G = g->g;
        if (method == 3) {
            return op.residual == PR_RES_FP32 ? solve_power_t<float>(G, p, op, pi, st)
                                              : solve_power_t<double>(G, p, op, pi, st);
        }
        const bool ifp2 = method == 2;
        return op.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, ifp2, p, -1, op, pi, st)
                                          : solve_ifp_t<double>(G, ifp2, p, -1, op, pi, st);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_state_create(int64_t n, const double *p, pr_state **out) {
    g_err.clear();
    if (!out) return fail(PR_EINVAL, "out is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(PR_EINVAL, "n must be in [1, 2^31)");
    std::vector<double> h((size_t)n, 1.0);
    if (p) {
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!(p[i] >= 0.0) || !std::isfinite(p[i])) return fail(PR_EINVAL, "p has a negative or non-finite entry");
            sum += p[i];
        }
        if (!(sum > 0.0)) return fail(PR_EINVAL, "p must have a positive sum");
        for (int64_t i = 0; i < n; ++i) h[(size_t)i] = (double)n * p[i] / sum;
    }
    std::unique_ptr<pr_state> S(new (std::nothrow) pr_state());
    if (!S) return fail(PR_ENOMEM, "host allocation");
    S->n = n;
    HIPCHK(hipGetDevice(&S->device));
    HIPCHK(hipMalloc((void **)&S->pibar, sizeof(double) * (size_t)n));
    HIPCHK(hipMalloc((void **)&S->h, sizeof(double) * (size_t)n));
    HIPCHK(hipMemset(S->pibar, 0, sizeof(double) * (size_t)n));
    HIPCHK(hipMemcpy(S->h, h.data(), sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    *out = S.release();
    return PR_OK;
}

pr_status pr_state_free(pr_state *s) {
    g_err.clear();
    if (!s) return PR_OK;
    (void)hipSetDevice(s->device);
    delete s;
    return PR_OK;
}

pr_status pr_state_read(const pr_state *s, double *pibar, double *h) {
    g_err.clear();
    if (!s) return fail(PR_EINVAL, "state is NULL");
    HIPCHK(hipSetDevice(s->device));
    if (pibar) HIPCHK(hipMemcpy(pibar, s->pibar, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost));
    if (h) HIPCHK(hipMemcpy(h, s->h, sizeof(double) * (size_t)s->n, hipMemcpyDeviceToHost));
    return PR_OK;
}

pr_status pr_solve_ifp2_warm(const pr_graph *g, const pr_opts *o, pr_state *s, double *pi, pr_stats *st) {
    g_err.clear();
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    if (!s) return fail(PR_EINVAL, "state is NULL");
    if (!pi) return fail(PR_EINVAL, "pi is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    if (op.flags & (PR_IFP2_LITERAL | PR_P_DEVICE)) return fail(PR_EINVAL, "option flag not supported for warm solves");
    if (g->g.n != s->n) return fail(PR_EINVAL, "graph and state differ in n");
    if (g->g.nP > 0) return fail(PR_EINVAL, "warm starts need a graph uploaded without PR_PEEL");
    if (s->c != 0.0 && s->c != op.c) return fail(PR_EINVAL, "c differs from the state's damping factor");
    ps = enter(g);
    if (ps != PR_OK) return ps;
    GraphUse use;
    ps = use_graph(g->g, use);
    if (ps != PR_OK) return ps;
    try {
        WarmArgs wa{s->pibar, s->h};
        ps = op.residual == PR_RES_FP32 ? solve_ifp_t<float>(g->g, true, nullptr, -1, op, pi, st, &wa)
                                        : solve_ifp_t<double>(g->g, true, nullptr, -1, op, pi, st, &wa);
        if (ps >= 0) s->c = op.c;
        return ps;
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_state_update(pr_state *s, const pr_graph *g_old, const pr_graph *g_new, const int32_t *changed,
                          int32_t k) {
    g_err.clear();
    if (!s || !g_old || !g_new) return fail(PR_EINVAL, "NULL argument");
    if (s->c == 0.0) return fail(PR_EINVAL, "the state has not been solved yet (no damping factor)");
    if (g_old->g.n != s->n || g_new->g.n != s->n) return fail(PR_EINVAL, "graphs and state differ in n");
    if (g_old->g.nP > 0 || g_new->g.nP > 0)
        return fail(PR_EINVAL, "warm starts need graphs uploaded without PR_PEEL");
    if (changed && k < 0) return fail(PR_EINVAL, "k < 0");
    if (changed)
        for (int32_t q = 0; q < k; ++q)
            if (changed[q] < 0 || changed[q] >= s->n) return fail(PR_EINVAL, "changed source out of [0, n)");
    HIPCHK(hipSetDevice(s->device));
    GraphUse use_old, use_new;
    pr_status ps = use_graph(g_old->g, use_old);
    if (ps == PR_OK) ps = use_graph(g_new->g, use_new);
    if (ps != PR_OK) return ps;
    hipStream_t st = g_new->g.stream;
    int32_t *d_src = nullptr;
    if (changed && k > 0) {
        HIPCHK(hipMalloc((void **)&d_src, sizeof(int32_t) * (size_t)k));
        HIPCHK(hipMemcpyAsync(d_src, changed, sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice, st));
    }
    struct Free {
        int32_t *p;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } fr{d_src};
    // both graphs' streams may still hold work that reads them
    HIPCHK(hipStreamSynchronize(g_old->g.stream));
    HIPCHK(launch_state_update(d_src, changed ? (int64_t)k : s->n, g_old->g, g_new->g, s->c, s->pibar, s->h, st));
    HIPCHK(hipStreamSynchronize(st));
    return PR_OK;
}

pr_status pr_graph_tune(pr_graph *g, const pr_opts *o, int32_t reps, pr_tune_report *rep) {
    g_err.clear();
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    if (op.flags & (PR_FORCE_PUSH | PR_FORCE_PULL | PR_FORCE_LIST | PR_P_DEVICE))
        return fail(PR_EINVAL, "tuning times the automatic schedule of global solves");
    ps = enter(g);
    if (ps != PR_OK) return ps;
    TuneLock lock;
    ps = lock_for_tuning(g->g, lock);
    if (ps != PR_OK) return ps;
    try {
        return tune_impl(g->g, op, reps, rep);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_set_upload(int32_t k, const int64_t *n, const int64_t *const *row_ptr, const int32_t *const *col,
                        uint32_t flags, pr_graph_set **out) {
    g_err.clear();
    try {
        return set_upload_impl(k, n, row_ptr, col, flags, out);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_set_free(pr_graph_set *s) {
    g_err.clear();
    if (!s) return PR_OK;
    (void)hipSetDevice(s->u->g.device);
    delete s;
    return PR_OK;
}

pr_status pr_set_info(const pr_graph_set *s, pr_set_info_t *out) {
    g_err.clear();
    if (!s || !out) return fail(PR_EINVAL, "NULL argument");
    const Graph &G = s->u->g;
    out->k = s->k;
    out->n = G.n;
    out->m = G.m;
    out->n_dangling = G.nD;
    out->m_dangling = G.mND;
    out->device_bytes = G.device_bytes + (int64_t)(2 * sizeof(int32_t) * ((size_t)s->k + 1));
    out->seconds_upload = G.seconds_upload;
    out->groups = s->ngr;
    out->tile_items = (int64_t)kBlock * G.tile_k;
    out->ordered = s->ngr > 1 && s->prefer_ordered ? 1 : 0;
    return PR_OK;
}

pr_status pr_set_tune(pr_graph_set *s, const double *c, const pr_opts *o, int32_t reps, pr_tune_report *rep) {
    g_err.clear();
    if (!s) return fail(PR_EINVAL, "graph set is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    if (c) op.c = 0.5;  // per-graph factors are checked by the solve
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    if (op.flags & (PR_FORCE_PUSH | PR_FORCE_PULL | PR_FORCE_LIST | PR_P_DEVICE | PR_IFP2_LITERAL | PR_PROFILE))
        return fail(PR_EINVAL, "tuning times the automatic schedule of set solves");
    ps = enter(s->u);
    if (ps != PR_OK) return ps;
    TuneLock lock;
    ps = lock_for_tuning(s->u->g, lock);
    if (ps != PR_OK) return ps;
    try {
        return set_tune_impl(*s, c, op, reps, rep);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_set_solve_ifp2(const pr_graph_set *s, const double *c, const pr_opts *o, double *pi, pr_stats *st) {
    g_err.clear();
    if (!s) return fail(PR_EINVAL, "graph set is NULL");
    if (!pi) return fail(PR_EINVAL, "pi is NULL");
    pr_opts op;
    opts_or_default(o, &op);
    if (c) op.c = 0.5;  // per-graph factors are checked by the solve
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    if (op.flags & (PR_P_DEVICE | PR_IFP2_LITERAL | PR_PROFILE | PR_VERIFY | PR_FORCE_LIST))
        return fail(PR_EINVAL, "option flag not supported for graph sets");
    ps = enter(s->u);
    if (ps != PR_OK) return ps;
    GraphUse use;
    ps = use_graph(s->u->g, use);
    if (ps != PR_OK) return ps;
    try {
        return op.residual == PR_RES_FP32 ? solve_set_t<float>(*s, c, op, pi, st)
                                          : solve_set_t<double>(*s, c, op, pi, st);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
}

pr_status pr_solve_ifp1(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st) {
    return solve_common(g, 1, p, o, pi, st);
}

pr_status pr_solve_ifp2(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st) {
    return solve_common(g, 2, p, o, pi, st);
}

pr_status pr_solve_power(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st) {
    return solve_common(g, 3, p, o, pi, st);
}

pr_status pr_ppr(const pr_graph *g, const int32_t *sources, int32_t k, const pr_opts *o, double *pi,
                 pr_stats *st) {
    g_err.clear();
    const int32_t fail_at = t_fail_ppr_batch;  // testing hook, one call only
    t_fail_ppr_batch = 0;
    if (!g) return fail(PR_EINVAL, "graph is NULL");
    if (!pi) return fail(PR_EINVAL, "pi is NULL");
    if (!sources || k < 1) return fail(PR_EINVAL, "need k >= 1 sources");
    const Graph &G = g->g;
    for (int32_t r = 0; r < k; ++r)
        if (sources[r] < 0 || sources[r] >= G.n) return fail(PR_EINVAL, "source out of [0, n)");
    pr_opts op;
    opts_or_default(o, &op);
    if (op.flags & PR_P_DEVICE) return fail(PR_EINVAL, "pr_ppr takes no p vector");
    pr_status ps = check_opts(op, false);
    if (ps != PR_OK) return ps;
    ps = enter(g);
    if (ps != PR_OK) return ps;
    GraphUse use;
    ps = use_graph(G, use);
    if (ps != PR_OK) return ps;
    pr_status worst = PR_OK;
    try {
        // groups of kBatch sources share one batched solve; a lone source runs alone, as
        // does every source on a peeled graph (the batched sweeps cover every non-dangling row)
        // (and with PR_VERIFY, whose check is part of the single-vector solve)
        const int32_t width = (G.nP > 0 || (op.flags & (PR_VERIFY | PR_FORCE_LIST))) ? 1 : kBatch;
        const int32_t nbatch = (k + width - 1) / width;
        const hipStream_t s = op.stream ? (hipStream_t)op.stream : G.stream;
        // more than one batch: every row is solved into device staging first and copied
        // out only once all batches have succeeded, so a failing batch writes no row
        DevBufs staging;
        double *stage = nullptr;
        pr_opts ob = op;
        if (nbatch > 1) {
            HIPCHK(staging.alloc(&stage, (size_t)k * (size_t)G.n));
            ob.flags |= PR_OUT_DEVICE;
        }
        std::vector<pr_stats> sts(st ? (size_t)k : 0);
        for (int32_t r = 0, b = 0; r < k; r += width, ++b) {
            if (fail_at > 0 && b == fail_at) return fail(PR_ENOMEM, "injected failure of a later batch (testing hook)");
            const int kb = (int)std::min<int32_t>(width, k - r);
            double *rows = (nbatch > 1 ? stage : pi) + (size_t)r * (size_t)G.n;
            pr_stats *sr = st ? sts.data() + r : nullptr;
            pr_status rs;
            if (kb == 1) {
                rs = ob.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, true, nullptr, sources[r], ob, rows, sr)
                                                : solve_ifp_t<double>(G, true, nullptr, sources[r], ob, rows, sr);
            } else if (kb <= 8) {
                rs = ob.residual == PR_RES_FP32 ? solve_ppr_batch_t<float, 8>(G, sources + r, kb, ob, rows, sr)
                                                : solve_ppr_batch_t<double, 8>(G, sources + r, kb, ob, rows, sr);
            } else {
                rs = ob.residual == PR_RES_FP32 ? solve_ppr_batch_t<float, 16>(G, sources + r, kb, ob, rows, sr)
                                                : solve_ppr_batch_t<double, 16>(G, sources + r, kb, ob, rows, sr);
            }
            if (rs < 0) return rs;
            if (rs > worst) worst = rs;
        }
        if (nbatch > 1) {
            const bool out_dev = op.flags & PR_OUT_DEVICE;
            HIPCHK(hipMemcpyAsync(pi, stage, sizeof(double) * (size_t)k * (size_t)G.n,
                                  out_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (st) std::copy(sts.begin(), sts.end(), st);
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
    return worst;
}

void pr_debug_fail_ppr_batch(int32_t b) { t_fail_ppr_batch = b > 0 ? b : 0; }

}  // extern "C"
