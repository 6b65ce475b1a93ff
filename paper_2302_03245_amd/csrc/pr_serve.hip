// pr_serve.hip -- query server of include/pr_serve.h: one engine (host thread +
// HIP stream + query workspace) per resident graph, query slots = columns of the
// batched solve, continuous admission and retirement between rounds, and
// workspaces taken against the server's memory budget per run.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pr_serve.h"
#include "pr_host.h"

using namespace prk;
using namespace prk::host;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct Request {
    int64_t id = 0;
    int32_t gid = 0;
    int32_t source = -1;
    double *out = nullptr;
    double t_submit = 0, t_done = 0;
    bool done = false;
    pr_status status = PR_OK;
    pr_stats st{};
    std::string err;
};

struct Engine;

}  // namespace

struct pr_server {
    pr_server_opts o{};
    std::mutex mu;
    std::condition_variable cv_done;
    std::vector<std::unique_ptr<Engine>> engines;
    std::unordered_map<int64_t, std::shared_ptr<Request>> reqs;
    int64_t next_id = 1;
    int64_t submitted = 0;
    std::vector<double> lat_ms;
    double edges_done = 0, t_first = -1, t_last = 0;
    // memory admission (guarded by mu)
    int64_t budget = 0;
    int64_t graph_bytes = 0;  // device bytes of the registered graphs
    int64_t ws_used = 0;      // query workspaces the engines hold
    int64_t max_single = 0;   // largest single-query workspace of a registered graph
    int64_t peak = 0;
    int64_t mem_waits = 0, narrowed = 0, rejected = 0;
    std::deque<Engine *> mem_queue;  // engines waiting for workspace memory, oldest first
    std::condition_variable cv_mem;
    std::atomic<bool> stop{false};
};

namespace {

struct Engine {
    pr_server *srv = nullptr;
    const pr_graph *hg = nullptr;
    const Graph *G = nullptr;
    int32_t gid = 0;
    int B = 16;  // widest batched run
    bool fp32 = true;
    hipStream_t stream = nullptr;
    char *ws = nullptr;    // query workspace, held between runs while no engine waits for memory
    size_t ws_bytes = 0;   // its size, counted in srv->ws_used
    bool wide_blocked = false;  // the last 16-wide workspace request found no room
    CtlB *hctl = nullptr;  // pinned
    std::deque<std::shared_ptr<Request>> queue;  // guarded by srv->mu
    std::condition_variable cv_work;
    std::thread th;
    bool holds_use = false;  // counted among the graph's users (no tuning while served)

    ~Engine() {
        if (th.joinable()) th.join();
        if (holds_use) {
            Graph &g = const_cast<Graph &>(*G);
            std::lock_guard<std::mutex> lk(g.ws_mu);
            --g.users;
        }
        if (ws) (void)hipFree(ws);
        if (hctl) (void)hipHostFree(hctl);
        if (stream) (void)hipStreamDestroy(stream);
    }

    // workspace of the batched runs (same carving for both residual types)
    static size_t footprint(const Graph &G, int B, bool fp32) {
        const size_t sT = fp32 ? 4 : 8;
        size_t b = 0;
        b += align256((size_t)G.n * B * sT);
        b += align256((size_t)G.nN * B * sT);
        b += align256((size_t)G.nN * B * 8);
        b += align256((size_t)std::max<int32_t>(G.nD, 1) * B * 8);
        b += align256((size_t)G.nN * B * 8);
        b += align256(sizeof(CtlB));
        b += align256(batch_part_doubles(B, batch_groups(G, B)) * 8);
        return b;
    }
    // vertex groups of the ordered sweeps of a batched run of width B (0: synchronous sweeps)
    static int batch_groups(const Graph &G, int B) {
        return batch_ordered_ready(G, B == 8 ? 0 : 1) ? (int)G.grp.size() - 1 : 0;
    }

    // workspace of a single-vector solve in this server's residual type
    size_t single_bytes() const {
        pr_opts o = single_opts();
        return fp32 ? solve_ifp_bytes<float>(*G, true, nullptr, o, false)
                    : solve_ifp_bytes<double>(*G, true, nullptr, o, false);
    }
    size_t width_bytes(int w) const { return w == 1 ? single_bytes() : footprint(*G, w, fp32); }
    pr_opts single_opts() const;
    enum class Room { held, none, failed };
    Room hold_ws(size_t need, std::string *err);
    void release_ws();
    void leave_mem_queue();  // caller holds srv->mu

    template <typename T>
    void serve();
    template <typename T, int Bw>
    bool run();
    template <typename T>
    bool run_single();
    bool trivial(const Request &r) const { return r.source >= 0 && G->dangling(r.source); }
    void take_trivial(std::vector<std::shared_ptr<Request>> &out);
    bool answer_trivial(std::vector<std::shared_ptr<Request>> &rs, bool sync);
    void finish(const std::shared_ptr<Request> &r, pr_status status, const pr_stats *st, const std::string &err);
};

void Engine::finish(const std::shared_ptr<Request> &r, pr_status status, const pr_stats *st,
                    const std::string &err) {
    const double tnow = now_s();
    std::lock_guard<std::mutex> lk(srv->mu);
    r->t_done = tnow;
    r->done = true;
    r->status = status;
    r->err = err;
    if (st) r->st = *st;
    else memset(&r->st, 0, sizeof(r->st));
    r->st.seconds_solve = tnow - r->t_submit;
    if (status >= 0) {
        srv->lat_ms.push_back((tnow - r->t_submit) * 1e3);
        srv->edges_done += (double)G->m;
        srv->t_last = std::max(srv->t_last, tnow);
    }
}

pr_opts Engine::single_opts() const {
    pr_opts o;
    pr_opts_default(&o);
    o.c = srv->o.c;
    o.l1_tol = srv->o.l1_tol;
    o.stop = PR_STOP_L1;
    o.residual = srv->o.residual;
    o.max_sweeps = srv->o.max_sweeps;
    o.flags = PR_OUT_DEVICE;
    o.stream = (void *)stream;
    return o;
}

void Engine::leave_mem_queue() {
    auto it = std::find(srv->mem_queue.begin(), srv->mem_queue.end(), this);
    if (it == srv->mem_queue.end()) return;
    srv->mem_queue.erase(it);
    srv->cv_mem.notify_all();
}

// Give the workspace back (its stream idle first): the memory and its share of the budget.
void Engine::release_ws() {
    if (!ws) return;
    (void)hipStreamSynchronize(stream);
    (void)hipFree(ws);
    ws = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->ws_used -= (int64_t)ws_bytes;
    ws_bytes = 0;
    srv->cv_mem.notify_all();
}

// Make the engine hold a workspace of at least `need` bytes: the one it holds if large enough,
// else a new one when the budget has room for it next to the registered graphs and the
// other engines' workspaces -- the engine's widest workspace when there is room for that
// (later runs of any width reuse it), else exactly `need`.  Engines waiting for memory
// take it in arrival order: one that does not hold enough gets memory only when no engine
// waits ahead of it.  Room::failed: the allocation itself failed with no other workspace
// to wait for (*err).
Engine::Room Engine::hold_ws(size_t need, std::string *err) {
    if (ws && ws_bytes >= need) return Room::held;
    const size_t old = ws_bytes;
    const size_t widest = std::max(need, std::max(width_bytes(B), single_bytes()));
    size_t bytes = need;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        const bool first = srv->mem_queue.empty() || srv->mem_queue.front() == this;
        const int64_t others = srv->graph_bytes + srv->ws_used - (int64_t)old;
        if (!first || others + (int64_t)need > srv->budget) return Room::none;
        if (others + (int64_t)widest <= srv->budget) bytes = widest;
        srv->ws_used += (int64_t)bytes - (int64_t)old;  // reserved before the memory is taken
        srv->peak = std::max(srv->peak, srv->graph_bytes + srv->ws_used);
    }
    if (ws) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(ws);
        ws = nullptr;
    }
    hipError_t e = hipMalloc((void **)&ws, bytes);
    if (e != hipSuccess && bytes > need) {  // the device refuses the widest: exactly what is needed
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->ws_used -= (int64_t)(bytes - need);
        }
        bytes = need;
        e = hipMalloc((void **)&ws, bytes);
    }
    if (e == hipSuccess) {
        ws_bytes = bytes;
        return Room::held;
    }
    (void)hipGetLastError();
    ws = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->ws_used -= (int64_t)bytes;
    ws_bytes = 0;
    srv->cv_mem.notify_all();
    // memory outside the budget is in use: wait while other workspaces may come back
    if (srv->ws_used > 0) return Room::none;
    *err = std::string("query workspace of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e);
    return Room::failed;
}

// A single-source query whose source has no out-edges needs no sweep: its
// PageRank is e_s exactly (no mass ever leaves s; the normalisation is 1).
// Such queries are taken out of the queue (caller holds srv->mu) ...
void Engine::take_trivial(std::vector<std::shared_ptr<Request>> &out) {
    for (auto it = queue.begin(); it != queue.end();) {
        if (trivial(**it)) {
            out.push_back(*it);
            it = queue.erase(it);
        } else {
            ++it;
        }
    }
}

// ... and answered with one fill each on the engine's stream (completed after
// the stream has been synchronised: here if sync, else by the caller).
bool Engine::answer_trivial(std::vector<std::shared_ptr<Request>> &rs, bool sync) {
    hipError_t e = hipSuccess;
    for (auto &r : rs)
        if (e == hipSuccess) e = launch_unit_vector(r->out, G->n, r->source, stream);
    if (sync && e == hipSuccess) e = hipStreamSynchronize(stream);
    if (!sync) return e == hipSuccess;
    pr_stats st{};
    for (auto &r : rs)
        finish(r, e == hipSuccess ? PR_OK : PR_EDEVICE, e == hipSuccess ? &st : nullptr,
               e == hipSuccess ? std::string() : std::string("fill: ") + hipGetErrorString(e));
    rs.clear();
    srv->cv_done.notify_all();
    return e == hipSuccess;
}

// Dispatcher of one engine: single-vector solves or batched runs, by queue length and by
// the workspace memory the budget allows: the width the queue asks for, else the widest
// narrower one that fits, else the queries wait until another engine gives memory back.
template <typename T>
void Engine::serve() {
    (void)hipSetDevice(G->device);
    bool ok = true;
    while (ok && !srv->stop.load()) {
        size_t q = 0;
        bool yield = false;  // another engine waits for memory ahead of this one
        std::vector<std::shared_ptr<Request>> triv;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            auto waits_ahead = [&] { return !srv->mem_queue.empty() && srv->mem_queue.front() != this; };
            cv_work.wait_for(lk, std::chrono::milliseconds(50),
                             [&] { return srv->stop.load() || !queue.empty() || (ws && waits_ahead()); });
            take_trivial(triv);
            q = queue.size();
            if (q == 0) leave_mem_queue();
            yield = ws && waits_ahead();
        }
        if (!triv.empty()) ok = answer_trivial(triv, true);
        if (yield) release_ws();
        if (!ok || q == 0 || srv->stop.load()) continue;
        const int want = (int64_t)q < (int64_t)srv->o.batch_min ? 1 : (B == 16 && q > 8 ? 16 : 8);
        int width = 0;
        Room room = Room::none;
        std::string err;
        for (int w = want; w >= 1; w = w == 8 ? 1 : w / 2) {
            room = hold_ws(width_bytes(w), &err);
            if (w == 16) wide_blocked = room != Room::held;
            if (room == Room::held) {
                width = w;
                break;
            }
        }
        if (room == Room::failed) {
            std::shared_ptr<Request> r;
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                leave_mem_queue();
                if (!queue.empty()) {
                    r = queue.front();
                    queue.pop_front();
                    ++srv->rejected;
                }
            }
            if (r) finish(r, PR_ENOMEM, nullptr, err);
            srv->cv_done.notify_all();
            continue;
        }
        if (width == 0) {  // wait for memory (engines ahead in the queue go first)
            std::unique_lock<std::mutex> lk(srv->mu);
            if (std::find(srv->mem_queue.begin(), srv->mem_queue.end(), this) == srv->mem_queue.end()) {
                srv->mem_queue.push_back(this);
                ++srv->mem_waits;
                for (auto &e : srv->engines) e->cv_work.notify_all();  // idle holders give memory back
            }
            srv->cv_mem.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            leave_mem_queue();
            if (width < want) ++srv->narrowed;
        }
        if (width == 1) ok = run_single<T>();
        else if (width == 16) ok = run<T, 16>();
        else ok = run<T, 8>();
        srv->cv_done.notify_all();
    }
    release_ws();
    std::lock_guard<std::mutex> lk(srv->mu);
    leave_mem_queue();
    for (auto &r : queue) {
        r->done = true;
        r->status = ok ? PR_EINVAL : PR_EDEVICE;
        r->err = ok ? "server destroyed" : "device error in this graph's engine";
    }
    queue.clear();
    srv->cv_done.notify_all();
}

// The oldest waiting query solved alone on the engine's stream, in the engine's workspace.
template <typename T>
bool Engine::run_single() {
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (queue.empty()) return true;
        r = queue.front();
        queue.pop_front();
    }
    const pr_opts o = single_opts();
    pr_stats st{};
    Ctl sctl;  // host copy of the control block
    ExtWorkspace ext{ws, ws_bytes, &sctl};
    pr_status ps;
    try {
        ps = solve_ifp_t<T>(*G, true, nullptr, r->source, o, r->out, &st, nullptr, &ext);
    } catch (const std::bad_alloc &) {
        ps = set_error(PR_ENOMEM, "host allocation");
    }
    finish(r, ps, ps >= 0 ? &st : nullptr, ps < 0 ? std::string(pr_last_error()) : std::string());
    srv->cv_done.notify_all();
    return ps != PR_EDEVICE;
}

// One batched run of residual type T and width Bw: lasts until its last column retires.
template <typename T, int Bw>
bool Engine::run() {
    const Graph &g = *G;
    hipStream_t s = stream;
    const int64_t n = g.n;
    const int32_t nN = g.nN, nD = g.nD;
    const double c = srv->o.c;
    const double tol = srv->o.l1_tol * (1.0 - 1e-6);
    const double xi = srv->o.l1_tol * (1.0 - c) / (2.0 * c) * (double)n / (double)std::max<int32_t>(nN, 1) *
                      (1.0 - 1e-9);
    const int S = srv->o.sweeps_per_round;
    const int max_sweeps = srv->o.max_sweeps > 0 ? srv->o.max_sweeps : 100000;
    const int slot = Bw == 8 ? 0 : 1;

    if (!ws || ws_bytes < footprint(g, Bw, fp32)) return false;  // the dispatcher holds it first
    char *p = ws;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return r;
    };
    T *h = (T *)take((size_t)n * Bw * sizeof(T));
    T *w = (T *)take((size_t)nN * Bw * sizeof(T));
    double *pibar = (double *)take((size_t)nN * Bw * 8);
    double *xD = (double *)take((size_t)std::max<int32_t>(nD, 1) * Bw * 8);
    double *w2 = (double *)take((size_t)nN * Bw * 8);
    CtlB *dctl = (CtlB *)take(sizeof(CtlB));
    // ordered sweeps once the frontier is dense (see solve_ppr_batch_t)
    const int ngr = batch_groups(g, Bw);
    const size_t part_n = batch_part_doubles(Bw, ngr);
    double *part = (double *)take(part_n * 8);
    double *sums = part + (part_n - (size_t)5 * Bw * ngr);
    const GroupBlocks gb = batch_group_blocks(g, Bw);

    std::shared_ptr<Request> slots[kMaxBatch];
    int t0[kMaxBatch] = {0};
    SrcSet ss;
    for (int j = 0; j < kMaxBatch; ++j) ss.s[j] = kSrcUnused;
    memset(hctl, 0, sizeof(CtlB));
    hctl->stop_after = INT_MAX;
    for (int j = 0; j < kMaxBatch; ++j) hctl->col_stop[j] = -1;
    int t = 0;
    bool ok = true;
    bool draining = false;
    std::string err;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && ok) {
            ok = false;
            err = std::string(what) + ": " + hipGetErrorString(e);
        }
        return e == hipSuccess;
    };

    while (!srv->stop.load()) {
        // ---- admission
        uint32_t admit = 0;
        int live = 0;
        std::vector<std::shared_ptr<Request>> triv;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            take_trivial(triv);
            int free_slots = 0;
            for (int j = 0; j < Bw; ++j) free_slots += slots[j] ? 0 : 1;
            // stop admitting: to restart 16 wide (when memory allows it), or to give the
            // workspace back to an engine that waits for memory
            if (Bw < B && !wide_blocked && (int)queue.size() > free_slots) draining = true;
            if (!srv->mem_queue.empty()) draining = true;
            for (int j = 0; j < Bw; ++j) {
                if (!draining && !slots[j] && !queue.empty()) {
                    slots[j] = queue.front();
                    queue.pop_front();
                    admit |= 1u << j;
                    t0[j] = t;
                }
                live += slots[j] ? 1 : 0;
            }
            if (live == 0 && triv.empty()) break;  // back to the dispatcher
        }
        if (live == 0) {
            if (!answer_trivial(triv, true)) {
                ok = false;
                err = "fill of single-source answers";
                break;
            }
            continue;
        }
        if (!triv.empty() && !answer_trivial(triv, false)) {
            ok = false;
            err = "fill of single-source answers";
        }
        if (admit) {
            for (int j = 0; j < Bw; ++j) {
                if (!((admit >> j) & 1u)) continue;
                ss.s[j] = slots[j]->source >= 0 ? slots[j]->source : kSrcUniform;
                hctl->col_stop[j] = INT_MAX;
                hctl->col_sweeps[j] = 0;
                hctl->sx[j] = (double)n;
                hctl->last_bound[j] = INFINITY;
                hctl->tot_pushes[j] = 0;
                hctl->tot_edges[j] = 0;
            }
            hctl->stop_after = INT_MAX;
            chk(hipMemcpyAsync(dctl, hctl, sizeof(CtlB), hipMemcpyHostToDevice, s), "control block");
            chk(launch_init_b<T, Bw>(n, nN, g.perm, ss, admit, h, pibar, s), "init");
        }
        // ---- a round of sweeps; the gather uses the epoch of the youngest live column
        int youngest = INT_MAX;
        for (int j = 0; j < Bw; ++j)
            if (slots[j]) youngest = std::min(youngest, t - t0[j]);
        const bool ordered = ngr > 1 && hctl->use_pull;  // the last decided sweep's frontier was dense
        for (int k = 0; k < S && ok && nN > 0; ++k, ++t, ++youngest) {
            size_t e = 0;
            while (e + 1 < g.epochs.size() && g.epochs[e + 1].t_start <= youngest) ++e;
            const MPPlan &pullp = g.bp_pull_nn[slot][e];
            const double pull_thr = kScatterShareBatch * (double)pullp.edges();
            if (ordered) {
                const std::vector<MPPlan> &gp = g.bp_grp[slot][e];
                unsigned long long sweep_edges = 0;
                for (int q = 0; q < ngr && ok; ++q) {
                    chk(launch_reserve_range_b<T, Bw>(t, dctl, g.grp[q], g.grp[q + 1], h, w, pibar, g.deg, g.rp_nn, c,
                                                      xi, g.bp_qle, gb.nb[q], part + (size_t)5 * Bw * kGroupBlocks * q,
                                                      s),
                        "reserve");
                    sweep_edges += (unsigned long long)gp[q].edges();
                    chk(launch_pull_b<T, T, Bw>(t, dctl, gp[q], w, h, 0, s), "pull");
                }
                chk(launch_decide_gs_b<Bw>(t, dctl, ngr, gb, part, sums, c, 1, tol, pull_thr, sweep_edges, s),
                    "decision");
                continue;
            }
            chk(launch_reserve_b<T, Bw>(t, dctl, nN, h, w, pibar, g.deg, g.rp_nn, c, xi, 1, tol, pull_thr, 0,
                                        (unsigned long long)pullp.edges(), part, s),
                "reserve");
            chk(launch_push_b<T, Bw>(t, dctl, g.bp_push_nn[slot], w, h, 1, s), "push");
            chk(launch_pull_b<T, T, Bw>(t, dctl, pullp, w, h, 1, s), "pull");
        }
        chk(hipMemcpyAsync(hctl, dctl, sizeof(CtlB), hipMemcpyDeviceToHost, s), "control block");
        chk(hipStreamSynchronize(s), "sweeps");
        if (!triv.empty()) {  // filled before this round's sweeps, on the same stream
            pr_stats st0{};
            for (auto &r : triv) finish(r, ok ? PR_OK : PR_EDEVICE, ok ? &st0 : nullptr, ok ? std::string() : err);
            triv.clear();
            srv->cv_done.notify_all();
        }
        // ---- retirement of the columns that met their bound (or ran out of sweeps)
        uint32_t fin = 0;
        OutSet os;
        for (int j = 0; j < kMaxBatch; ++j) os.p[j] = nullptr;
        for (int j = 0; j < Bw; ++j) {
            if (!slots[j]) continue;
            if (!ok || nN == 0 || hctl->col_stop[j] < t || t - t0[j] >= max_sweeps) {
                fin |= 1u << j;
                os.p[j] = slots[j]->out;
            }
        }
        if (!fin) continue;
        if (ok && nD > 0) chk(launch_phase2_b<T, Bw>(n, nN, g.perm, ss, h, pibar, g.deg, c, w2, xD, g.bp_pull_nd[slot], s),
                              "dangling phase");
        if (ok) chk(launch_final_b<T, Bw>(dctl, n, nN, g.perm, fin, os, h, pibar, xD, part, s), "normalisation");
        if (ok) chk(hipMemcpyAsync(hctl, dctl, sizeof(CtlB), hipMemcpyDeviceToHost, s), "control block");
        if (ok) chk(hipStreamSynchronize(s), "normalisation");
        for (int j = 0; j < Bw; ++j) {
            if (!((fin >> j) & 1u)) continue;
            if (!ok) {
                finish(slots[j], PR_EDEVICE, nullptr, err);
            } else {
                pr_stats st{};
                const bool conv = hctl->col_stop[j] < t || nN == 0;
                st.sweeps = hctl->col_sweeps[j];
                st.edges_processed = (int64_t)hctl->tot_edges[j] + g.mND;
                st.vertex_pushes = (int64_t)hctl->tot_pushes[j];
                const double fs = hctl->fin_sum[j];
                st.residual_l1 = fs > 0 ? hctl->fin_sn[j] / fs : 0.0;
                st.l1_bound = fs > 0 ? 2.0 * c / (1.0 - c) * hctl->fin_sn[j] / fs : 0.0;
                st.seconds_preprocess = g.seconds_split;
                finish(slots[j], conv ? PR_OK : PR_ENOCONV, &st, std::string());
            }
            slots[j].reset();
            ss.s[j] = kSrcUnused;
            hctl->col_stop[j] = -1;
        }
        // the host copy of the control block stays authoritative for the next admission
        srv->cv_done.notify_all();
        if (!ok) break;
    }
    // columns still live here: the server is being destroyed, or the device failed
    std::lock_guard<std::mutex> lk(srv->mu);
    for (int j = 0; j < Bw; ++j) {
        if (!slots[j]) continue;
        slots[j]->done = true;
        slots[j]->status = ok ? PR_EINVAL : PR_EDEVICE;
        slots[j]->err = ok ? "server destroyed" : err;
    }
    return ok;
}

}  // namespace

extern "C" {

void pr_server_opts_default(pr_server_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->c = 0.85;
    o->l1_tol = 1e-6;
    o->residual = PR_RES_FP32;
    o->slots = 16;
    o->batch_min = 2;
    o->sweeps_per_round = 4;
}

pr_status pr_server_create(const pr_server_opts *o, pr_server **out) {
    clear_error();
    if (!out) return set_error(PR_EINVAL, "out is NULL");
    pr_server_opts op;
    if (o) op = *o;
    else pr_server_opts_default(&op);
    if (!(op.c > 0.0 && op.c < 1.0)) return set_error(PR_EINVAL, "c must be in (0, 1)");
    if (!(op.l1_tol > 0.0) || !isfinite(op.l1_tol)) return set_error(PR_EINVAL, "l1_tol must be > 0 and finite");
    if (op.residual != PR_RES_FP32 && op.residual != PR_RES_FP64) return set_error(PR_EINVAL, "unknown residual type");
    if (op.slots != 8 && op.slots != 16) return set_error(PR_EINVAL, "slots must be 8 or 16");
    if (op.sweeps_per_round < 1) return set_error(PR_EINVAL, "sweeps_per_round must be >= 1");
    if (op.batch_min < 1) return set_error(PR_EINVAL, "batch_min must be >= 1");
    if (op.max_sweeps < 0 || op.memory_budget < 0) return set_error(PR_EINVAL, "negative limit");
    std::unique_ptr<pr_server> sv(new (std::nothrow) pr_server());
    if (!sv) return set_error(PR_ENOMEM, "host allocation");
    sv->o = op;
    if (op.memory_budget > 0) {
        sv->budget = op.memory_budget;
    } else {
        size_t fr = 0, tot = 0;
        hipError_t e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) return set_error(PR_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
        sv->budget = (int64_t)(0.9 * (double)tot);
    }
    *out = sv.release();
    return PR_OK;
}

pr_status pr_server_add_graph(pr_server *s, const pr_graph *g, int32_t *graph_id) {
    clear_error();
    if (!s || !g || !graph_id) return set_error(PR_EINVAL, "NULL argument");
    const Graph &G = g->g;
    if (G.nP > 0) return set_error(PR_EINVAL, "the server needs graphs uploaded without PR_PEEL");
    const bool fp32 = s->o.residual == PR_RES_FP32;
    std::unique_ptr<Engine> eng(new (std::nothrow) Engine());
    if (!eng) return set_error(PR_ENOMEM, "host allocation");
    eng->srv = s;
    eng->hg = g;
    eng->G = &G;
    eng->B = s->o.slots;
    eng->fp32 = fp32;
    // the graph and one query's workspace must fit next to the graphs already registered
    // (workspaces held by running engines come and go and are not counted here)
    auto fits = [&](int64_t gbytes, const char *when) {
        const int64_t one = (int64_t)eng->single_bytes();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->graph_bytes + gbytes + std::max(s->max_single, one) > s->budget)
            return set_error(PR_ENOMEM, std::string("the graph and one query's workspace exceed the server's memory budget") +
                                            when + " (" + std::to_string(s->graph_bytes + gbytes) + " + " +
                                            std::to_string(std::max(s->max_single, one)) + " > " +
                                            std::to_string(s->budget) + " bytes)");
        return PR_OK;
    };
    pr_status ps = fits(G.device_bytes, "");
    if (ps != PR_OK) return ps;
    {
        Graph &gm = const_cast<Graph &>(G);
        std::lock_guard<std::mutex> lk(gm.ws_mu);
        if (gm.tuning) return set_error(PR_EBUSY, "the graph is being tuned");
        ++gm.users;
        eng->holds_use = true;
    }
    hipError_t e = hipSetDevice(G.device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&eng->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return set_error(PR_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
    // batch plans and the stop rule's weights stay on the graph
    for (int bw = 8; bw <= eng->B; bw *= 2) {
        ps = batch_plans(const_cast<Graph &>(G), bw, eng->stream);
        if (ps != PR_OK) return set_error(ps, "batch plans");
    }
    ps = host::stop_weights(const_cast<Graph &>(G), s->o.c, eng->stream);
    if (ps != PR_OK) return ps;
    const int64_t gbytes = G.device_bytes;
    ps = fits(gbytes, " with its batch plans");
    if (ps != PR_OK) return ps;
    e = hipHostMalloc((void **)&eng->hctl, sizeof(CtlB), hipHostMallocDefault);
    if (e != hipSuccess) return set_error(PR_ENOMEM, "pinned control block");
    Engine *ep = eng.get();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->graph_bytes += gbytes;
        s->max_single = std::max(s->max_single, (int64_t)ep->single_bytes());
        s->peak = std::max(s->peak, s->graph_bytes + s->ws_used);
        ep->gid = (int32_t)s->engines.size();
        s->engines.push_back(std::move(eng));
    }
    ep->th = std::thread(ep->fp32 ? &Engine::serve<float> : &Engine::serve<double>, ep);
    *graph_id = ep->gid;
    return PR_OK;
}

pr_status pr_server_footprint(pr_server *s, int32_t graph_id, int32_t width, int64_t *bytes) {
    clear_error();
    if (!s || !bytes) return set_error(PR_EINVAL, "NULL argument");
    if (width != 1 && width != 8 && width != 16) return set_error(PR_EINVAL, "width must be 1, 8 or 16");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->engines.size()) return set_error(PR_EINVAL, "unknown graph id");
    *bytes = (int64_t)s->engines[(size_t)graph_id]->width_bytes(width);
    return PR_OK;
}

pr_status pr_server_submit(pr_server *s, int32_t graph_id, int32_t source, double *pi_device, int64_t *request_id) {
    clear_error();
    if (!s || !pi_device || !request_id) return set_error(PR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->engines.size()) return set_error(PR_EINVAL, "unknown graph id");
    Engine &eng = *s->engines[(size_t)graph_id];
    if (source < -1 || source >= eng.G->n) return set_error(PR_EINVAL, "source out of [-1, n)");
    auto r = std::make_shared<Request>();
    r->id = s->next_id++;
    r->gid = graph_id;
    r->source = source;
    r->out = pi_device;
    r->t_submit = now_s();
    if (s->t_first < 0) s->t_first = r->t_submit;
    s->reqs[r->id] = r;
    s->submitted += 1;
    eng.queue.push_back(r);
    eng.cv_work.notify_one();
    *request_id = r->id;
    return PR_OK;
}

pr_status pr_server_wait(pr_server *s, int64_t request_id, double timeout_seconds, pr_stats *st) {
    clear_error();
    if (!s) return set_error(PR_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return set_error(PR_EINVAL, "unknown or already collected request");
    std::shared_ptr<Request> r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_seconds < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_seconds), pred)) {
        return set_error(PR_EDEVICE, "timeout");
    }
    s->reqs.erase(it);
    if (st) *st = r->st;
    if (r->status < 0) return set_error(r->status, r->err);
    return r->status;
}

pr_status pr_server_get_stats(pr_server *s, pr_server_stats *out) {
    clear_error();
    if (!s || !out) return set_error(PR_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = (int64_t)s->lat_ms.size();
    out->device_bytes = s->graph_bytes + s->ws_used;
    out->graph_bytes = s->graph_bytes;
    out->peak_bytes = s->peak;
    out->budget = s->budget;
    out->memory_waits = s->mem_waits;
    out->narrowed_runs = s->narrowed;
    out->rejected = s->rejected;
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto q = [&](double f) { return v[(size_t)std::min<double>((double)v.size() - 1, floor(f * (double)v.size()))]; };
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        out->max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
        const double span = s->t_last - s->t_first;
        out->edges_per_second = span > 0 ? s->edges_done / span : 0.0;
    }
    return PR_OK;
}

pr_status pr_server_destroy(pr_server *s) {
    clear_error();
    if (!s) return PR_OK;
    s->stop.store(true);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &e : s->engines) e->cv_work.notify_all();
        s->cv_mem.notify_all();
    }
    for (auto &e : s->engines)
        if (e->th.joinable()) e->th.join();
    s->engines.clear();
    delete s;
    return PR_OK;
}

}  // extern "C"
