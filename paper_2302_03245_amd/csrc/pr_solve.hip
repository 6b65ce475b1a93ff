// pr_solve.hip -- the sweep loops of libpr.so's solvers (IFP1, IFP2, the power
// method, batched PPR columns), their workspaces, and the per-graph autotuner.
#include "pr_host.h"

namespace prk {
namespace host {

pr_status acquire_ws(Graph &G, size_t bytes, Workspace &ws, hipStream_t s) {
    ws.g = &G;
    ws.bytes = bytes;
    ws.stream = s;
    {
        std::lock_guard<std::mutex> lk(G.ws_mu);
        if (!G.ws_busy) {
            if (G.ws_bytes < bytes) {
                if (G.ws_mem) (void)hipFree(G.ws_mem);
                G.ws_mem = nullptr;
                G.ws_bytes = 0;
                hipError_t e = hipMalloc(&G.ws_mem, bytes);
                if (e != hipSuccess) return hip_fail(e, "workspace");
                G.ws_bytes = bytes;
            }
            if (!G.ws_hctl) {
                hipError_t e = hipHostMalloc(&G.ws_hctl, sizeof(Ctl), hipHostMallocDefault);
                if (e != hipSuccess) return hip_fail(e, "pinned control block");
            }
            G.ws_busy = true;
            ws.base = (char *)G.ws_mem;
            ws.hctl = (Ctl *)G.ws_hctl;
            ws.cached = true;
            return PR_OK;
        }
    }
    hipError_t e = hipMalloc((void **)&ws.base, bytes);
    if (e != hipSuccess) return hip_fail(e, "workspace");
    e = hipHostMalloc((void **)&ws.hctl, sizeof(Ctl), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned control block");
    return PR_OK;
}


// Error weights of IFP2's stop rule for damping factor c (see ErrWeights): built once per
// graph and factor on the solve's stream and kept on the graph (for up to kMaxAmp
// factors; a solve that may not allocate, or finds the table full, keeps the uniform
// weight c / (1 - c)).  kAmpIters iterations of the recursion leave the weights within
// about c^k of their limit on the graphs measured (the residual decays at the rate of
// c P restricted to the non-dangling vertices).
constexpr int kMaxAmp = 4;
constexpr int kAmpIters = 16;

static pr_status amp_weights(Graph &G, double c, bool may_alloc, hipStream_t s, ErrWeights *out,
                             double *seconds = nullptr) {
    *out = ErrWeights{nullptr, nullptr};
    if (seconds) *seconds = 0.0;
    std::lock_guard<std::mutex> lk(G.amp_mu);
    for (const Graph::Amp &a : G.amp)
        if (a.c == c) {
            *out = ErrWeights{a.g, a.q};
            if (seconds) *seconds = a.seconds;
            return PR_OK;
        }
    if (!may_alloc || (int)G.amp.size() >= kMaxAmp || G.nN == 0 || G.mNN == 0) return PR_OK;
    const auto t0 = std::chrono::steady_clock::now();
    DevBufs tmp;
    double *f = nullptr, *acc = nullptr;
    HIPCHK(tmp.alloc(&f, (size_t)G.nN));
    HIPCHK(tmp.alloc(&acc, (size_t)G.nN));
    DevBufs keep;
    float *g = nullptr, *q = nullptr;
    HIPCHK(keep.alloc(&g, (size_t)G.nN));
    HIPCHK(keep.alloc(&q, (size_t)G.nN));
    HIPCHK(launch_amp_weights(G.nN, G.push_nn, G.deg, G.rp_nn, c, kAmpIters, f, acc, g, q, s));
    HIPCHK(hipStreamSynchronize(s));  // other streams may take the weights from the table
    for (void *p : keep.ptrs) {
        G.allocs.push_back(p);
        G.device_bytes += (int64_t)sizeof(float) * G.nN;
    }
    keep.ptrs.clear();
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    G.amp.push_back(Graph::Amp{c, g, q, sec});
    *out = ErrWeights{g, q};
    if (seconds) *seconds = sec;
    return PR_OK;
}

// The push weights of ordered sweeps restricted to each vertex's own and earlier groups
// (launch_amp_qle) for factor c and the graph's current vertex groups, built on first use
// and kept with the factor's weights; null when the factor has no weights, or when they
// are missing and the solve may not allocate (the sweeps then sum S_N directly).
static pr_status amp_qle(Graph &G, double c, bool may_alloc, hipStream_t s, const float **out, double *seconds) {
    *out = nullptr;
    *seconds = 0.0;
    const int32_t ng = (int32_t)G.grp.size() - 1;
    if (ng < 2 || ng > kMaxGroups) return PR_OK;
    std::lock_guard<std::mutex> lk(G.amp_mu);
    for (Graph::Amp &a : G.amp) {
        if (a.c != c) continue;
        if (a.qle && a.qle_version == G.grp_version) {
            *out = a.qle;
            *seconds = a.qle_seconds;
            return PR_OK;
        }
        if (!may_alloc) return PR_OK;
        if (!a.qle) {
            DevBufs keep;
            float *q = nullptr;
            HIPCHK(keep.alloc(&q, (size_t)G.nN));
            G.allocs.push_back((void *)q);
            G.device_bytes += (int64_t)sizeof(float) * G.nN;
            keep.ptrs.clear();
            a.qle = q;
        }
        GroupEnds ge{};
        ge.ng = ng;
        for (int32_t q = 0; q < ng; ++q) ge.end[q] = G.grp[(size_t)q + 1];
        const auto t0 = std::chrono::steady_clock::now();
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(launch_amp_qle(G.nN, G.rp_nn, G.col_nn, G.deg, a.g, ge, a.qle, s));
        HIPCHK(hipStreamSynchronize(s));  // other streams may take the weights from the table
        a.qle_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        a.qle_version = G.grp_version;
        *out = a.qle;
        *seconds = a.qle_seconds;
        return PR_OK;
    }
    return PR_OK;
}

// The stop rule's error weights for factor c built ahead of solves that may not allocate
// (a server engine's solves run in a workspace of its own).
pr_status stop_weights(Graph &G, double c, hipStream_t s) {
    ErrWeights ew;
    return amp_weights(G, c, true, s, &ew);
}

// Validate p (host or device) and place it on the device; returns 1/sum(p).
pr_status prepare_p(const Graph &G, const double *p, const pr_opts &o, double *pdev, double *sumbad,
                    const double **p_used, double *pscale, hipStream_t s) {
    *p_used = nullptr;
    *pscale = 1.0;
    if (!p) return PR_OK;
    double sum = 0.0;
    if (o.flags & PR_P_DEVICE) {
        HIPCHK(launch_zero_f64(sumbad, 2, s));
        HIPCHK(launch_validate_p(p, G.n, sumbad, s));
        double h[2];
        HIPCHK(hipMemcpyAsync(h, sumbad, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[1] != 0.0) return fail(PR_EINVAL, "p has a negative or non-finite entry");
        sum = h[0];
        *p_used = p;
    } else {
        for (int64_t i = 0; i < G.n; ++i) {
            if (!(p[i] >= 0.0) || !isfinite(p[i])) return fail(PR_EINVAL, "p has a negative or non-finite entry");
            sum += p[i];
        }
        HIPCHK(hipMemcpyAsync(pdev, p, sizeof(double) * G.n, hipMemcpyHostToDevice, s));
        *p_used = pdev;
    }
    if (!(sum > 0.0) || !isfinite(sum)) return fail(PR_EINVAL, "sum(p) must be > 0");
    *pscale = 1.0 / sum;
    return PR_OK;
}

// Sweep batches: the kernels of sweeps past the stop decision return at once,
// so the host enqueues a batch, reads the control block, and sizes the next
// batch from the observed decay of the certified bound.
int next_batch(int prev_batch, double bound_prev, double bound_now, int swept, double tol, bool l1) {
    if (l1 && bound_prev > 0 && bound_now > 0 && bound_now < bound_prev && swept > 0) {
        double rate = pow(bound_now / bound_prev, 1.0 / swept);
        if (rate > 0 && rate < 1) {
            // past the target (the threshold rule's tail, where a few residuals stay
            // above xi): grow the batch again, but by at most 16 sweeps
            if (bound_now <= tol) return std::min(16, std::max(2, prev_batch * 2));
            const double need = log(tol / bound_now) / log(rate);
            int k = (int)ceil(need) + 1;
            return std::min(64, std::max(2, k));
        }
    }
    return std::min(64, prev_batch * 2);
}

// A-posteriori check of a written result (PR_VERIFY): one application of P'' (Eq. 1)
// to the normalised output in FP64 (the vertices with out-edges are [0, nN + nP)).
// The copy of the control block is read back with the solve's own (same stream).
// g: the stop rule's weights for factor c (null: the check without row weights)
static hipError_t run_verify(const Graph &G, const InitArgs &a, double c, const float *g, const double *out, double *x,
                             double *acc, double *y, Ctl *vctl, double *part, Ctl *res, double *depth, hipStream_t s) {
    Ctl hc;
    memset(&hc, 0, sizeof(hc));
    hc.stop_after = INT_MAX;
    hipError_t e = hipMemcpyAsync(vctl, &hc, sizeof(Ctl), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    InitArgs av = a;
    av.nN = G.nN + G.nP;
    e = launch_verify(vctl, av, out, x, acc, y, G.deg, G.pull_all, G.in_ptr, c, g, G.nN, G.rp_nn, part, depth, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(res, vctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// ||pi - pi_exact||_1 <= ||P'' pi - pi||_1 / (1 - c) + |sum(pi) - 1| (P'' contracts by c
// the differences of vectors with equal sums), and with row weights f (weighted)
// <= 2 sum_j f_j |r_j| / sum(pi) + |sum(pi) - 1| (see launch_verify); the smaller of the
// two, each FP64 quantity widened by the rounding of its own computation (unit roundoff
// 2^-53, first order, with 1 % margin; a row's weight is at most 1 / (1 - c))
static double verified_bound(const Ctl &v, double depth, double c, bool weighted) {
    const double u = ldexp(1.0, -53) * 1.01;
    const double tail = fabs(v.ver_sum - 1.0) + depth * u * v.ver_sum;
    const double r = v.ver_r * (1.0 + depth * u) + v.ver_err * u;
    double best = r / (1.0 - c) + tail;
    if (weighted && v.ver_sum > 0.0) {
        const double rf = std::min(v.ver_rf, v.ver_rf2) * (1.0 + depth * u) + v.ver_err * u / (1.0 - c);
        best = std::min(best, 2.0 * rf / (v.ver_sum * (1.0 - depth * u)) + tail);
    }
    return best;
}

// PR_VERIFY under the L1 rule: rounds of further sweeps when the check finds the result
// short of the target; the device stop flag is reopened from this constant
constexpr int kVerifyRounds = 3;
static const int kNoStop = INT_MAX;

// Workspace layout of solve_ifp_t (the order of the carve below).
template <typename T>
size_t solve_ifp_bytes(const Graph &G, bool ifp2, const double *p, const pr_opts &o, bool warm) {
    (void)ifp2;
    const int64_t n = G.n;
    const int32_t nN = G.nN, nD = G.nD;
    const bool out_dev = o.flags & PR_OUT_DEVICE;
    const bool verify = o.flags & PR_VERIFY;
    const bool list_ok = !warm && !(o.flags & (PR_FORCE_PUSH | PR_FORCE_PULL)) && nN > 0;
    const int64_t wave_cap = (int64_t)nN + ((int64_t)G.mNN + G.mND) / kChunkEdges + 1;
    const size_t list_bytes = list_ok ? 3 * carve_size<int32_t>(nN) + carve_size<T>(nN) +
                                            2 * carve_size<int32_t>(wave_cap) + carve_size<T>(wave_cap)
                                      : 0;
    return list_bytes + (verify ? 2 * carve_size<double>(n) + carve_size<Ctl>(1) : 0) +
           carve_size<T>(n) + carve_size<T>(nN) + carve_size<double>(nN) + carve_size<double>(nD) +
           carve_size<double>(nN + G.nP) + carve_size<double>(out_dev ? 0 : n) + carve_size<Ctl>(1) +
           carve_size<Trace>(1) + carve_size<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0) +
           carve_size<double>(2) + carve_size<double>(kPartDoubles) +
           (warm ? 2 * carve_size<double>(nN) + 3 * carve_size<double>(nD) : 0);
}

template <typename T>
pr_status solve_ifp_t(const Graph &G, bool ifp2, const double *p, int32_t source, const pr_opts &o, double *pi,
                      pr_stats *st, const WarmArgs *warm, const ExtWorkspace *ext) {
    hipStream_t s = o.stream ? (hipStream_t)o.stream : G.stream;
    const int64_t n = G.n;
    const int32_t nN = G.nN, nD = G.nD;
    const bool literal = ifp2 && (o.flags & PR_IFP2_LITERAL);
    const bool out_dev = o.flags & PR_OUT_DEVICE;
    const double c = o.c;
    const bool l1 = o.stop == PR_STOP_L1;
    // threshold: under the L1 rule, the xi at which an empty frontier already
    // certifies the bound (residual on N <= nN * xi, total mass >= n)
    double xi = o.xi;
    if (l1) {
        xi = o.l1_tol * (1.0 - c) / (2.0 * c) * (double)n / (double)std::max<int32_t>(nN, 1);
        xi *= 1.0 - 1e-9;
    }
    const double tol = l1 ? o.l1_tol * (1.0 - 1e-6) : 0.0;
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 100000;
    const int64_t launches0 = t_kernel_launches;
    const bool verify = o.flags & PR_VERIFY;
    // list sweeps (compacted frontier) need non-negative residuals: not for warm starts
    const bool force_list = o.flags & PR_FORCE_LIST;
    const bool list_ok = !warm && !(o.flags & (PR_FORCE_PUSH | PR_FORCE_PULL)) && nN > 0;
    const int64_t wave_cap = (int64_t)nN + ((int64_t)G.mNN + G.mND) / kChunkEdges + 1;
    const size_t bytes = solve_ifp_bytes<T>(G, ifp2, p, o, warm != nullptr);
    Workspace ws;
    pr_status ps = PR_OK;
    if (ext) {
        if (bytes > ext->bytes) return fail(PR_EINVAL, "workspace larger than the memory provided");
        ws.base = (char *)ext->base;
        ws.bytes = bytes;
        ws.hctl = ext->hctl;
        ws.stream = s;
        ws.borrowed = true;
    } else {
        ps = acquire_ws(const_cast<Graph &>(G), bytes, ws, s);
        if (ps != PR_OK) return ps;
    }
    Carve cv{ws.base};
    T *h = cv.take<T>(n);
    T *w = cv.take<T>(nN);
    double *pibar = cv.take<double>(nN);
    double *xD = cv.take<double>(nD);
    double *w2 = cv.take<double>(nN + G.nP);  // phase-2 weights of every source of a deferred vertex
    double *outbuf = cv.take<double>(out_dev ? 0 : n);
    Ctl *ctl = cv.take<Ctl>(1);
    Trace *tr = cv.take<Trace>(1);
    double *pdev = cv.take<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0);
    double *sumbad = cv.take<double>(2);
    double *part = cv.take<double>(kPartDoubles);
    // warm start: reserve at the start, mass taken this solve pushed to dangling vertices
    double *pibar0 = warm ? cv.take<double>(nN) : nullptr;
    double *w3 = warm ? cv.take<double>(nN) : nullptr;
    double *xD0 = warm ? cv.take<double>(nD) : nullptr;
    double *hD0 = warm ? cv.take<double>(nD) : nullptr;
    double *hDn = warm ? cv.take<double>(nD) : nullptr;
    double *vx = verify ? cv.take<double>(n) : nullptr;
    double *vacc = verify ? cv.take<double>(n) : nullptr;
    Ctl *vctl = verify ? cv.take<Ctl>(1) : nullptr;
    ListBufs<T> lb{};
    if (list_ok) {
        lb.f[0] = cv.take<int32_t>(nN);
        lb.f[1] = cv.take<int32_t>(nN);
        lb.lane_v = cv.take<int32_t>(nN);
        lb.lane_w = cv.take<T>(nN);
        lb.wave_v = cv.take<int32_t>(wave_cap);
        lb.wave_c = cv.take<int32_t>(wave_cap);
        lb.wave_w = cv.take<T>(wave_cap);
    }

    InitArgs a{};
    a.n = n;
    a.nN = nN;
    a.perm = G.perm;
    a.source = source;
    a.uniform = (p == nullptr && source < 0);
    ps = prepare_p(G, p, o, pdev, sumbad, &a.p, &a.pscale, s);
    if (ps != PR_OK) return ps;
    // the stop rule's error bound: per-vertex weights for folded IFP2 on a graph without
    // peeled vertices (the weighted sum bounds the unnormalised error itself, so the
    // factor is 2 for the normalisation), else c / (1 - c) per unit of residual.  A warm
    // start takes them only when the graph already has them: after a change the graph is
    // new, and building them (a few gathers over its edges) would cost a large share of
    // the few sweeps a warm start needs
    ErrWeights ew{nullptr, nullptr};
    double seconds_weights = 0.0;
    if (ifp2 && !literal && G.nP == 0) {
        ps = amp_weights(const_cast<Graph &>(G), c, ext == nullptr && !warm, s, &ew, &seconds_weights);
        if (ps != PR_OK) return ps;
    }
    const double kb = ew.g ? 2.0 : 2.0 * c / (1.0 - c);

    EventPair ev_solve(ext == nullptr);  // no events in a solve that allocates nothing
    SweepTimer timer;
    timer.on = o.flags & PR_PROFILE;
    if (ev_solve.a) HIPCHK(hipEventRecord(ev_solve.a, s));
    Ctl hc;
    memset(&hc, 0, sizeof(hc));
    hc.stop_after = INT_MAX;
    hc.sx = (double)n;
    HIPCHK(hipMemcpyAsync(ctl, &hc, sizeof(Ctl), hipMemcpyHostToDevice, s));
    if (warm)
        HIPCHK(launch_warm_import<T>(ctl, n, nN, G.perm, warm->pibar, warm->h, h, pibar, pibar0, xD0, hD0, part, s));
    else
        HIPCHK(launch_init_ifp<T>(a, h, pibar, s));

    // the gather of sweep t uses the in-edge lists of the last epoch starting at or before t
    auto pull_plan = [&](int t) -> const MPPlan & {
        size_t e = 0;
        while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
        return ifp2 ? G.epochs[e].pull_nn : G.epochs[e].pull_all;
    };
    const int force = (o.flags & PR_FORCE_PUSH) ? 1 : ((o.flags & PR_FORCE_PULL) ? 2 : 0);
    const int check_mode = force == 0;
    // ordered sweeps (groups built at upload): from the start for global solves, where every
    // vertex starts active; otherwise from the first batch after a sweep that gathered.  IFP2
    // gathers into the non-dangling rows, IFP1 into all rows (its pushes reach dangling vertices)
    const int ngr = (int)G.grp.size() - 1;
    const bool ordered_ok = ngr > 1 && ngr <= kMaxGroups && force == 0 && !(o.flags & PR_JACOBI) &&
                            !G.grp_pull.empty() && G.prefer_ordered;
    // ordered sweeps with the stop rule's weights take S_N from the reserves' own sums,
    // with the pushed mass weighted by the part that stays residual to the end of a sweep
    // (no summing pass per sweep); residuals of either sign (a warm start) are summed
    const float *qle = nullptr;
    if (ordered_ok && ew.g && !warm) {
        double seconds_qle = 0.0;
        ps = amp_qle(const_cast<Graph &>(G), c, ext == nullptr, s, &qle, &seconds_qle);
        if (ps != PR_OK) return ps;
        seconds_weights += seconds_qle;  // built once per graph, factor and grouping: preprocessing
    }
    const ErrWeights ew_ord = qle ? ErrWeights{ew.g, qle} : ErrWeights{nullptr, nullptr};
    bool ordered = ordered_ok && a.uniform && !warm;
    GroupBlocks gb{};
    gb.stride = kGroupBlocks;
    for (int q = 0; q < ngr && q < kMaxGroups; ++q)
        gb.nb[q] = (int32_t)std::min<int64_t>(
            kGroupBlocks, std::max<int64_t>(1, ((int64_t)G.grp[q + 1] - G.grp[q] + 1023) / 1024));
    const double sT = (double)sizeof(T);
    int t = 0;
    bool stopped = false;
    // list sweeps: from the start when forced or for a single-source solve (its frontier
    // is one vertex); otherwise entered when a synchronous sweep's frontier has fewer valid
    // edges than kListShare of a gather's, and left when it (or the next frontier's
    // expected edges) grows past that
    bool list_on = list_ok && (force_list || (source >= 0 && !ordered));
    bool list_ready = false;
    // a solve that may turn to ordered sweeps checks its frontier after two sweeps
    int batch = (ordered_ok && !ordered) ? 2 : (l1 ? 8 : 16);
    double bound_prev = -1.0;
    int t_prev = 0;
    // the stop rule's target: tol, tightened when PR_VERIFY's check finds the result short
    double tol_run = tol;
    auto run_sweeps = [&]() -> pr_status {
        if (nN > 0) {
            while (t < max_sweeps) {
                if (list_on && !list_ready) {
                    // the list of sweep t from the residuals; counters of both parities cleared
                    HIPCHK(launch_zero_u32(&ctl->fcnt[0], 8, s));
                    HIPCHK(launch_zero_u32((uint32_t *)(void *)&ctl->fedges[0], 4, s));
                    HIPCHK(launch_compact<T>(ctl, t & 1, nN, h, xi, lb.f[t & 1], G.deg, G.rp_nn, ifp2 ? 1 : 0,
                                             ew.g, part, s));
                    list_ready = true;
                }
                // while sparse, the host looks at the frontier after every sweep (it can grow a
                // hundredfold in one: a hub enters it)
                const int bmax = (list_on && !force_list) ? 1 : batch;
                int nb = std::min(bmax, max_sweeps - t);
                // a batch that starts after a dense sweep gathers throughout (a gather is right
                // for any frontier) and launches no scatter that would only exit at once
                const int sweep_force =
                    (force == 0 && t > 0 &&
                     (double)ws.hctl->last_edges >= kScatterShare * (double)pull_plan(t).edges())
                        ? 2
                        : force;
                for (int k = 0; k < nb; ++k, ++t) {
                    if (list_on) {
                        HIPCHK(launch_reserve_list<T>(t, ctl, tr, lb, h, pibar, G.deg, G.rp_nn, c, xi, ifp2 ? 1 : 0, ew,
                                                      kb, l1 ? 1 : 0, tol_run, part, s));
                        HIPCHK(launch_push_list<T>(t, ctl, lb, h, G.deg, G.rp_nn, G.col_nn, G.rp_nd, G.col_nd, xi,
                                                   ifp2 ? 1 : 0, s));
                        continue;
                    }
                    const MPPlan &pullp = pull_plan(t);
                    // a gather reads every live in-edge; scatter while the active edges are a
                    // smaller share of them than kScatterShare
                    const unsigned long long pull_edges = (unsigned long long)pullp.edges();
                    const unsigned long long pull_thr = (unsigned long long)(kScatterShare * (double)pull_edges) + 1;
                    if (ordered) {
                        size_t e = 0;
                        while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
                        unsigned long long sweep_edges = 0;
                        for (int q = 0; q < ngr; ++q) {
                            HIPCHK(launch_reserve_range<T>(t, ctl, G.grp[q], G.grp[q + 1], h, w, pibar, G.deg,
                                                           G.rp_nn, c, xi, ifp2 ? 1 : 0, gb.nb[q], ew_ord,
                                                           part + (size_t)5 * kGroupBlocks * q, s));
                            const MPPlan &pl = G.group_rows ? (ifp2 ? G.grp_pull_rows[e][q] : G.grp_pull_all_rows[e][q])
                                                            : (ifp2 ? G.grp_pull[e][q] : G.grp_pull_all[e][q]);
                            sweep_edges += (unsigned long long)pl.edges();
                            // the method's own bytes: every gathered in-edge (source id + weight), and
                            // each target row once per sweep (offset + residual update), shared
                            // evenly by the group gathers
                            const double rows = ifp2 ? (double)nN : (double)n;
                            const KernelEvents ev = timer.next(
                                t, 1, (double)pl.edges() * (4.0 + sT) + rows * (4.0 + 2.0 * sT) / (double)ngr);
                            HIPCHK(launch_pull<T, T>(t, ctl, pl, w, h, 0, s, TileSkip(), ev));
                        }
                        HIPCHK(launch_decide_gs<T>(t, ctl, tr, nN, h, ngr, gb, part,
                                                   part + (size_t)5 * kGroupBlocks * ngr, c, ew.g, kb, l1 ? 1 : 0,
                                                   tol_run, pull_thr, sweep_edges, qle ? 1 : 0, s));
                        continue;
                    }
                    HIPCHK(launch_reserve<T>(t, ctl, tr, nN, h, w, pibar, G.deg, G.rp_nn, c, xi, ifp2 ? 1 : 0, ew, kb,
                                             l1 ? 1 : 0, tol_run, pull_thr, sweep_force, pull_edges, part, s));
                    if (sweep_force != 2) {
                        // the scatter is timed when it is forced; in the automatic mode only the
                        // gather (the dense sweeps' kernel) carries events, to keep their overhead low
                        const KernelEvents e = force == 1 ? timer.next(t, 0, 0.0) : KernelEvents();
                        if (ifp2) {
                            HIPCHK(launch_push<T>(t, ctl, G.push_nn, w, h, check_mode, s, TileSkip(), e));
                        } else {  // one interval over both scatter launches
                            HIPCHK(launch_push<T>(t, ctl, G.push_nn, w, h, check_mode, s, TileSkip(), {e.a, nullptr}));
                            HIPCHK(launch_push<T>(t, ctl, G.push_nd, w, h, check_mode, s, TileSkip(), {nullptr, e.b}));
                        }
                    }
                    if (force != 1) {
                        // every live in-edge: source id + gathered weight; every target row: offset + residual update
                        const KernelEvents e =
                            timer.next(t, 1, (double)pullp.edges() * (4.0 + sT) + (double)pullp.R * (4.0 + 2.0 * sT));
                        HIPCHK(launch_pull<T, T>(t, ctl, pullp, w, h, check_mode, s, TileSkip(), e));
                    }
                }
                HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (ws.hctl->stop_after < t) {
                    stopped = true;
                    break;
                }
                if (list_ok && !force_list) {
                    const double list_thr = kListShare * (double)pull_plan(t).edges();
                    if (list_on) {
                        // the valid out-edges of the frontier list of sweep t
                        const double next_edges = (double)ws.hctl->fedges[t & 1];
                        if ((double)ws.hctl->last_edges >= list_thr || next_edges >= list_thr) {
                            list_on = false;  // dense from the next sweep: its reserve reads every residual
                            list_ready = false;
                        }
                    } else if (!ordered && (double)ws.hctl->last_edges < list_thr) {
                        list_on = true;  // the list is built from the residuals before the next sweep
                    }
                }
                ordered = ordered_ok && ws.hctl->use_pull && !list_on;  // dense frontier: ordered sweeps from here
                // under the threshold rule the frontier empties some sweeps after the mean
                // residual on N reaches xi: the bound at that mean is the target of the sizing
                const double target = l1 ? tol_run : 2.0 * c / (1.0 - c) * xi * (double)nN / std::max(ws.hctl->sx, 1.0);
                batch = next_batch(batch, bound_prev, ws.hctl->last_bound, t - t_prev, target, true);
                // until the frontier is dense enough for ordered sweeps, look at it every two
                // sweeps (a long run of synchronous sweeps would forgo their faster decay)
                if (ordered_ok && !ordered) batch = std::min(batch, 2);
                bound_prev = ws.hctl->last_bound;
                t_prev = t;
            }
        } else {
            stopped = true;
        }
        return PR_OK;
    };
    ps = run_sweeps();
    if (ps != PR_OK) return ps;
    double *dst = out_dev ? pi : outbuf;
    // phase 2 and the normalised result from the current state
    auto finish = [&]() -> pr_status {
        if (ifp2 && nD > 0 && warm) {
            HIPCHK(launch_warm_phase2_prep<T>(nN, nD, h, pibar, pibar0, G.deg, c, xD0, hD0, w2, w3, xD, hDn, s));
            HIPCHK(launch_pull<double, double>(-1, ctl, G.pull_nd, w2, xD, 0, s));
            HIPCHK(launch_pull<double, double>(-1, ctl, G.pull_nd, w3, hDn, 0, s));
        } else if (ifp2 && G.nP > 0) {
            // peeled levels from the highest down: each gathers from the core and the levels
            // above it, then hands its own weights to the levels below; the dangling block last
            HIPCHK(launch_phase2_prep<T>(a, h, pibar, G.deg, c, literal ? 1 : 0, w2, xD, s));
            for (size_t b = 0; b < G.lvl_pull.size(); ++b) {
                const int32_t lo = G.lvl_lo[b], hi = G.lvl_lo[b + 1];
                HIPCHK(launch_pull<double, double>(-1, ctl, G.lvl_pull[b], w2, xD + (lo - nN), 0, s));
                if (lo < nN + G.nP) HIPCHK(launch_peel_w2(lo, hi, nN, xD, G.deg, c, w2, s));
            }
        } else if (ifp2 && nD > 0) {
            HIPCHK(launch_phase2_prep<T>(a, h, pibar, G.deg, c, literal ? 1 : 0, w2, xD, s));
            HIPCHK(launch_pull<double, double>(-1, ctl, G.pull_nd, w2, xD, 0, s));
        }
        HIPCHK(launch_final_ifp<T>(ctl, a, h, pibar, xD, ifp2 ? 1 : 0, literal ? 1 : 0, ew.g, dst, part, s));
        if (ev_solve.b) HIPCHK(hipEventRecord(ev_solve.b, s));
        return PR_OK;
    };
    ps = finish();
    if (ps != PR_OK) return ps;
    Ctl vres;
    double vdepth = 0.0;
    double l1_verified = 0.0;
    // the check's row weights: those of the stop rule (graphs without peeled vertices,
    // whose dangling vertices are the only absorbing ones)
    ErrWeights evw = ew;
    if (verify && !evw.g && G.nP == 0) {
        ps = amp_weights(const_cast<Graph &>(G), c, ext == nullptr, s, &evw);
        if (ps != PR_OK) return ps;
    }
    if (verify) {
        HIPCHK(run_verify(G, a, c, evw.g, dst, vx, vacc, w2, vctl, part, &vres, &vdepth, s));
        l1_verified = verified_bound(vres, vdepth, c, evw.g != nullptr);
        // Under the L1 rule the check can find the result short of the target when the
        // rounding of the sweeps (FP32 residuals) adds to the residual the stop rule
        // sees: sweep on to a target tighter by what the check adds, and check again
        const double kfin = literal ? 2.0 / (1.0 - c) : kb;
        int round = 0;
        while (l1 && !warm && stopped && l1_verified > o.l1_tol && t < max_sweeps && round++ < kVerifyRounds) {
            HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const double est = ws.hctl->fin_sum > 0 ? kfin * ws.hctl->fin_sn / ws.hctl->fin_sum : 0.0;
            const double room = o.l1_tol - (l1_verified - est);
            if (!(room > 0.0)) break;  // the check's excess alone exceeds the target
            tol_run = std::min(tol_run, room) * 0.9;
            HIPCHK(hipMemcpyAsync(&ctl->stop_after, &kNoStop, sizeof(int), hipMemcpyHostToDevice, s));
            stopped = false;
            ps = run_sweeps();
            if (ps != PR_OK) return ps;
            ps = finish();
            if (ps != PR_OK) return ps;
            HIPCHK(run_verify(G, a, c, evw.g, dst, vx, vacc, w2, vctl, part, &vres, &vdepth, s));
            l1_verified = verified_bound(vres, vdepth, c, evw.g != nullptr);
        }
    }
    if (warm) HIPCHK(launch_warm_export<T>(n, nN, G.perm, h, pibar, hDn, warm->pibar, warm->h, s));
    HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (!out_dev) HIPCHK(hipMemcpyAsync(pi, outbuf, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Ctl &r = *ws.hctl;
    if (st) {
        pr_stats z;
        memset(&z, 0, sizeof(z));
        z.sweeps = r.sweeps;
        z.pull_sweeps = r.pull_sweeps;
        z.edges_processed = (int64_t)r.tot_edges + (ifp2 ? G.mND : 0);
        z.edges_traversed = (int64_t)r.tot_traversed + (ifp2 ? G.mND : 0);
        z.vertex_pushes = (int64_t)r.tot_pushes;
        z.residual_l1 = r.fin_sum > 0 ? r.fin_res / r.fin_sum : 0.0;
        const double k = literal ? 2.0 / (1.0 - c) : kb;
        z.l1_bound = r.fin_sum > 0 ? k * r.fin_sn / r.fin_sum : 0.0;
        if (warm) {
            // signed residuals: unnormalised error E <= c / (1 - c) sum|h_N| (or the weighted
            // sum), the exact mass is at least fin_sum - E, and normalising costs
            // (1 + sum|x| / sum x) E / (that mass)
            const double E = 0.5 * kb * r.fin_sn;
            const double den = r.fin_sum - E;
            z.l1_bound = den > 0 ? (1.0 + r.fin_abs / r.fin_sum) * E / den : INFINITY;
        }
        z.seconds_solve = ev_solve.a ? elapsed_s(ev_solve.a, ev_solve.b) : 0.0;
        z.seconds_preprocess = ifp2 ? G.seconds_split + seconds_weights : 0.0;
        z.launches = t_kernel_launches - launches0;
        z.l1_verified = l1_verified;
        if (timer.on) {
            std::vector<unsigned long long> trc((size_t)std::min(r.sweeps + 1, kMaxTrace));
            std::vector<unsigned long long> tre(trc.size());
            std::vector<double> trs(trc.size()), trb(trc.size());
            if (!trc.empty()) {
                HIPCHK(hipMemcpy(trc.data(), tr->cnt, sizeof(unsigned long long) * trc.size(), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(tre.data(), tr->edges, sizeof(unsigned long long) * tre.size(),
                                 hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(trs.data(), tr->sn, sizeof(double) * trs.size(), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(trb.data(), tr->bound, sizeof(double) * trb.size(), hipMemcpyDeviceToHost));
            }
            g_trace = TraceRec();
            for (size_t i = 0; i < trc.size() && (int)i < r.sweeps; ++i) {
                g_trace.active.push_back((int64_t)(trc[i] & ~(1ull << 63)));
                g_trace.pulled.push_back((int32_t)(trc[i] >> 63));
                g_trace.edges.push_back((int64_t)tre[i]);
                g_trace.residual.push_back(trs[i]);
                g_trace.bound.push_back(trb[i]);
            }
            const double sT = (double)sizeof(T);
            for (size_t i = 0; i < timer.ev.size(); ++i) {
                int ts = timer.sweep_of[i];
                if (ts >= r.sweeps || ts >= (int)trc.size()) continue;
                bool pulled = (trc[ts] >> 63) != 0;
                if ((int)pulled != timer.is_pull[i]) continue;
                double sec = elapsed_s(timer.ev[i]->a, timer.ev[i]->b);
                if (sec <= 0.0) continue;  // nothing was launched (empty plan)
                if (pulled) {
                    z.pull_seconds += sec;
                    z.pull_launches += 1;
                    z.pull_bytes += timer.bytes[i];
                } else {
                    // every pushed edge: target id + residual read-modify-write; every row: offset + weight
                    int rows = ifp2 ? nN : 2 * nN;
                    z.push_seconds += sec;
                    z.push_launches += ifp2 ? 1 : 2;
                    z.push_bytes += (double)tre[ts] * (4.0 + 2.0 * sT) + (double)rows * (4.0 + sT);
                }
            }
        }
        *st = z;
    }
    if (verify && l1 && l1_verified > o.l1_tol) return PR_ENOCONV;
    return stopped ? PR_OK : PR_ENOCONV;
}

template <typename WT>
pr_status solve_power_t(const Graph &G, const double *p, const pr_opts &o, double *pi, pr_stats *st) {
    hipStream_t s = o.stream ? (hipStream_t)o.stream : G.stream;
    const int64_t n = G.n;
    const int32_t nN = G.nN + G.nP;  // vertices with out-edges (on a peeled graph, the core and the peeled ones)
    const bool out_dev = o.flags & PR_OUT_DEVICE;
    const double c = o.c;
    const double tol = o.l1_tol * (1.0 - 1e-6);
    const int max_it = o.max_sweeps > 0 ? o.max_sweeps : 100000;
    const int64_t launches0 = t_kernel_launches;
    const bool verify = o.flags & PR_VERIFY;
    size_t bytes = (verify ? carve_size<double>(nN) + carve_size<Ctl>(1) : 0) +
                   carve_size<double>(n) * 2 + carve_size<WT>(nN) + carve_size<double>(out_dev ? 0 : n) +
                   carve_size<Ctl>(1) + carve_size<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0) +
                   carve_size<double>(2) + carve_size<double>(5 * kRedBlocks);
    Workspace ws;
    pr_status ps = acquire_ws(const_cast<Graph &>(G), bytes, ws, s);
    if (ps != PR_OK) return ps;
    Carve cv{ws.base};
    double *x = cv.take<double>(n);
    double *acc = cv.take<double>(n);
    WT *y = cv.take<WT>(nN);
    double *outbuf = cv.take<double>(out_dev ? 0 : n);
    Ctl *ctl = cv.take<Ctl>(1);
    double *pdev = cv.take<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0);
    double *sumbad = cv.take<double>(2);
    double *part = cv.take<double>(5 * kRedBlocks);
    double *vy = verify ? cv.take<double>(nN) : nullptr;
    Ctl *vctl = verify ? cv.take<Ctl>(1) : nullptr;
    InitArgs a{};
    a.n = n;
    a.nN = nN;
    a.perm = G.perm;
    a.source = -1;
    a.uniform = p == nullptr;
    ps = prepare_p(G, p, o, pdev, sumbad, &a.p, &a.pscale, s);
    if (ps != PR_OK) return ps;

    EventPair ev_solve;
    SweepTimer timer;
    timer.on = o.flags & PR_PROFILE;
    HIPCHK(hipEventRecord(ev_solve.a, s));
    Ctl hc;
    memset(&hc, 0, sizeof(hc));
    hc.stop_after = INT_MAX;
    HIPCHK(hipMemcpyAsync(ctl, &hc, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIPCHK(launch_power_init(a, x, acc, s));
    int t = 0;
    bool stopped = false;
    int batch = 8;
    double bound_prev = -1.0;
    int t_prev = 0;
    while (t <= max_it) {
        int nb = std::min(batch, max_it + 1 - t);
        for (int k = 0; k < nb; ++k, ++t) {
            HIPCHK(launch_power_prescale<WT>(t, ctl, a, x, acc, y, G.deg, c, tol, part, s));
            if (t < max_it) {
                const KernelEvents e = timer.next(t, 1, 0.0);
                HIPCHK(launch_pull<WT, double>(t, ctl, G.pull_all, y, acc, 0, s, TileSkip(), e));
            }
        }
        HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ws.hctl->stop_after < t) {
            stopped = true;
            break;
        }
        batch = next_batch(batch, bound_prev, ws.hctl->last_bound, t - t_prev, tol, true);
        bound_prev = ws.hctl->last_bound;
        t_prev = t;
    }
    double *dst = out_dev ? pi : outbuf;
    HIPCHK(launch_final_x(ctl, a, x, dst, part, s));
    HIPCHK(hipEventRecord(ev_solve.b, s));
    Ctl vres;
    double vdepth = 0.0;
    // the iterate buffers are free once the answer is written: the check reuses them
    ErrWeights evw{nullptr, nullptr};
    if (verify && G.nP == 0) {
        ps = amp_weights(const_cast<Graph &>(G), c, true, s, &evw);
        if (ps != PR_OK) return ps;
    }
    if (verify) HIPCHK(run_verify(G, a, c, evw.g, dst, x, acc, vy, vctl, part, &vres, &vdepth, s));
    HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (!out_dev) HIPCHK(hipMemcpyAsync(pi, outbuf, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Ctl &r = *ws.hctl;
    const double l1_verified = verify ? verified_bound(vres, vdepth, c, evw.g != nullptr) : 0.0;
    if (st) {
        pr_stats z;
        memset(&z, 0, sizeof(z));
        z.sweeps = r.sweeps;
        z.pull_sweeps = r.sweeps;
        z.edges_processed = (int64_t)r.sweeps * G.m;
        z.edges_traversed = z.edges_processed;
        z.vertex_pushes = (int64_t)r.sweeps * nN;
        z.residual_l1 = r.pw_diff;
        z.l1_bound = c / (1.0 - c) * r.pw_diff;
        z.seconds_solve = elapsed_s(ev_solve.a, ev_solve.b);
        z.launches = t_kernel_launches - launches0;
        z.l1_verified = l1_verified;
        if (timer.on) {
            const double sW = (double)sizeof(WT);
            for (size_t i = 0; i < timer.ev.size(); ++i) {
                if (timer.sweep_of[i] >= r.sweeps) continue;
                z.pull_seconds += elapsed_s(timer.ev[i]->a, timer.ev[i]->b);
                z.pull_launches += 1;
                z.pull_bytes += (double)G.m * (4.0 + sW) + (double)n * (4.0 + 16.0);
            }
        }
        *st = z;
    }
    if (verify && l1_verified > o.l1_tol) return PR_ENOCONV;
    return stopped ? PR_OK : PR_ENOCONV;
}

// Ordered sweeps of the batched kernels of width B for the graph's current vertex groups:
// the groups' gathers over the rows they reach with tiles of (kBlock / B) * kMPK items,
// and the unit-weight qle of the sweeps' S_N bookkeeping.  Owned with the groups (freed
// and rebuilt with them); the caller holds bp_mu.
template <int B>
pr_status ensure_batch_groups(Graph &G, hipStream_t s) {
    constexpr int slot = B == 8 ? 0 : 1;
    const int32_t ng = (int32_t)G.grp.size() - 1;
    if (ng < 2 || ng > kMaxGroups || G.grp_pull_rows.size() != G.epochs.size()) return PR_OK;
    if (G.bp_grp_version[slot] == G.grp_version && (int)G.bp_grp[slot].size() == (int)G.epochs.size()) return PR_OK;
    auto galloc = [&](auto **p, size_t count) -> hipError_t {
        using U = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        *p = nullptr;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(U);
        hipError_t e = hipMalloc((void **)p, bytes);
        if (e == hipSuccess) {
            G.grp_allocs.push_back((void *)*p);
            G.grp_bytes += (int64_t)bytes;
            G.device_bytes += (int64_t)bytes;
        }
        return e;
    };
    if (G.bp_qle_version != G.grp_version || !G.bp_qle) {
        float *q = nullptr;
        HIPCHK(galloc(&q, (size_t)G.nN));
        GroupEnds ge{};
        ge.ng = ng;
        for (int32_t k = 0; k < ng; ++k) ge.end[k] = G.grp[(size_t)k + 1];
        HIPCHK(launch_amp_qle(G.nN, G.rp_nn, G.col_nn, G.deg, nullptr, ge, q, s));
        G.bp_qle = q;
        G.bp_qle_version = G.grp_version;
    }
    std::vector<std::vector<MPPlan>> plans;
    for (const std::vector<MPPlan> &ep : G.grp_pull_rows) {
        std::vector<MPPlan> row;
        for (const MPPlan &g1 : ep) {
            MPPlan p = g1;  // the same lists and rows, batched tiles
            p.ipb = (kBlock / B) * kMPK;
            p.blocks = 0;
            const int32_t blocks = (int32_t)(((int64_t)p.items + p.ipb - 1) / p.ipb);
            HIPCHK(galloc(&p.plan, (size_t)blocks + 1));
            if (p.R > 0) HIPCHK(launch_plan(p, s));
            row.push_back(p);
        }
        plans.push_back(row);
    }
    HIPCHK(hipStreamSynchronize(s));
    G.bp_grp[slot] = plans;
    G.bp_grp_version[slot] = G.grp_version;
    return PR_OK;
}

// Plans for the batched kernels of width B (tiles of (kBlock / B) * kMPK items),
// built once per graph and width on the first batched solve.
template <int B>
pr_status ensure_batch_plans_impl(Graph &G, hipStream_t s) {
    constexpr int slot = B == 8 ? 0 : 1;
    std::lock_guard<std::mutex> lk(G.bp_mu);
    // without room for the groups' batched plans, batches sweep synchronously
    auto groups = [&]() -> pr_status {
        const pr_status gs = ensure_batch_groups<B>(G, s);
        if (gs != PR_ENOMEM) return gs;
        (void)hipGetLastError();  // the refused allocation must not read as a later launch's error
        clear_error();
        return PR_OK;
    };
    if (G.bp_ready[slot]) return groups();
    auto mk = [&](MPPlan &p, const uint32_t *rpp, const int32_t *idx, int32_t R, int64_t edges) -> hipError_t {
        p.rp = rpp;
        p.idx = idx;
        p.R = R;
        p.items = (uint32_t)(R + edges);
        p.ipb = (kBlock / B) * kMPK;
        p.blocks = 0;
        const int32_t blocks = (int32_t)(((int64_t)p.items + p.ipb - 1) / p.ipb);
        void *mem = nullptr;
        hipError_t e = hipMalloc(&mem, sizeof(uint2) * ((size_t)blocks + 1));
        if (e != hipSuccess) return e;
        G.allocs.push_back(mem);
        G.device_bytes += (int64_t)(sizeof(uint2) * ((size_t)blocks + 1));
        p.plan = (uint2 *)mem;
        if (R == 0) return hipSuccess;
        return launch_plan(p, s);
    };
    G.bp_pull_nn[slot].clear();
    for (const Epoch &e : G.epochs) {
        MPPlan p;
        HIPCHK(mk(p, e.in_ptr, e.in_src, G.nN, e.edges_nn));
        G.bp_pull_nn[slot].push_back(p);
    }
    HIPCHK(mk(G.bp_pull_nd[slot], G.in_ptr + G.nN, G.in_src, G.nD, G.mND));
    HIPCHK(mk(G.bp_push_nn[slot], G.rp_nn, G.col_nn, G.nN, G.mNN));
    HIPCHK(hipStreamSynchronize(s));
    G.bp_ready[slot] = true;
    return groups();
}

// IFP2 for kb <= kBatch single-source PPR queries at once (pr_batch.hip):
// column-interleaved residuals, per-column management, one gather serving all
// columns.  pi_rows[r * n ...] receives the vector of srcs[r].
template <typename T, int B>
pr_status solve_ppr_batch_t(const Graph &Gc, const int32_t *srcs, int kb, const pr_opts &o, double *pi_rows,
                            pr_stats *st) {
    constexpr int slot = B == 8 ? 0 : 1;
    Graph &G = const_cast<Graph &>(Gc);
    // the batched dangling phase gathers from the swept vertices only: on a graph with
    // peeled vertices, whose in-edges into the deferred region also start at peeled
    // vertices, it would read past the swept vertices' weights
    if (G.nP > 0) return set_error(PR_EINVAL, "batched solves need a graph uploaded without PR_PEEL");
    hipStream_t s = o.stream ? (hipStream_t)o.stream : G.stream;
    pr_status ps = ensure_batch_plans_impl<B>(G, s);
    if (ps != PR_OK) return ps;
    const int64_t n = G.n;
    const int32_t nN = G.nN, nD = G.nD;
    const bool out_dev = o.flags & PR_OUT_DEVICE;
    const double c = o.c;
    const bool l1 = o.stop == PR_STOP_L1;
    double xi = o.xi;
    if (l1) xi = o.l1_tol * (1.0 - c) / (2.0 * c) * (double)n / (double)std::max<int32_t>(nN, 1) * (1.0 - 1e-9);
    const double tol = l1 ? o.l1_tol * (1.0 - 1e-6) : 0.0;
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 100000;

    const int force = (o.flags & PR_FORCE_PUSH) ? 1 : ((o.flags & PR_FORCE_PULL) ? 2 : 0);
    // ordered sweeps (the vertex groups' gathers one after another, each group reserving
    // after the earlier groups' gathers of the same sweep) once the frontier is dense
    const bool ordered_ok = force == 0 && !(o.flags & PR_JACOBI) && nN > 0 && batch_ordered_ready(G, slot);
    const int ngr = ordered_ok ? (int)G.grp.size() - 1 : 0;
    const size_t part_n = batch_part_doubles(B, ngr);
    size_t bytes = carve_size<T>((size_t)n * B) + carve_size<T>((size_t)nN * B) + carve_size<double>((size_t)nN * B) +
                   carve_size<double>((size_t)nD * B) + carve_size<double>((size_t)nN * B) +
                   carve_size<double>(out_dev ? 0 : (size_t)kb * n) + carve_size<CtlB>(1) + carve_size<double>(part_n);
    Workspace ws;
    ps = acquire_ws(G, bytes, ws, s);
    if (ps != PR_OK) return ps;
    Carve cv{ws.base};
    T *h = cv.take<T>((size_t)n * B);
    T *w = cv.take<T>((size_t)nN * B);
    double *pibar = cv.take<double>((size_t)nN * B);
    double *xD = cv.take<double>((size_t)nD * B);
    double *w2 = cv.take<double>((size_t)nN * B);
    double *outbuf = cv.take<double>(out_dev ? 0 : (size_t)kb * n);
    CtlB *ctl = cv.take<CtlB>(1);
    double *part = cv.take<double>(part_n);
    double *sums = part + (part_n - (size_t)5 * B * ngr);  // an ordered sweep's row sums
    const GroupBlocks gb = batch_group_blocks(G, B);
    CtlB *hc = nullptr;
    HIPCHK(hipHostMalloc((void **)&hc, sizeof(CtlB), hipHostMallocDefault));
    std::unique_ptr<CtlB, void (*)(CtlB *)> hc_guard(hc, [](CtlB *p) { (void)hipHostFree(p); });

    SrcSet ss;
    for (int j = 0; j < kMaxBatch; ++j) ss.s[j] = j < kb ? srcs[j] : -1;
    memset(hc, 0, sizeof(CtlB));
    hc->stop_after = INT_MAX;
    for (int j = 0; j < B; ++j) {
        hc->col_stop[j] = j < kb ? INT_MAX : -1;
        hc->sx[j] = (double)n;
    }
    EventPair ev_solve;
    HIPCHK(hipEventRecord(ev_solve.a, s));
    HIPCHK(hipMemcpyAsync(ctl, hc, sizeof(CtlB), hipMemcpyHostToDevice, s));
    const uint32_t kmask = (uint32_t)((1ull << kb) - 1ull);
    HIPCHK(launch_init_b<T, B>(n, nN, G.perm, ss, kmask, h, pibar, s));

    const int check_mode = force == 0;
    auto epoch_of = [&](int t) {
        size_t e = 0;
        while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
        return e;
    };
    auto pull_plan = [&](int t) -> const MPPlan & { return G.bp_pull_nn[slot][epoch_of(t)]; };
    int t = 0;
    bool stopped = false;
    if (nN > 0) {
        // single-source columns start with a frontier of one vertex each: synchronous
        // sweeps (scatters) first, the host looking every two sweeps for a dense frontier
        bool ordered = false;
        int batch = ordered_ok ? 2 : (l1 ? 8 : 16);
        double bound_prev = -1.0;
        int t_prev = 0;
        while (t < max_sweeps) {
            const int nbt = std::min(batch, max_sweeps - t);
            for (int k = 0; k < nbt; ++k, ++t) {
                const MPPlan &pullp = pull_plan(t);
                // a gather serves every column; scatter when the active (vertex, column) edges are few
                const double pull_thr = kScatterShareBatch * (double)pullp.edges();
                if (ordered) {
                    const std::vector<MPPlan> &gp = G.bp_grp[slot][epoch_of(t)];
                    unsigned long long sweep_edges = 0;
                    for (int q = 0; q < ngr; ++q) {
                        HIPCHK((launch_reserve_range_b<T, B>(t, ctl, G.grp[q], G.grp[q + 1], h, w, pibar, G.deg,
                                                             G.rp_nn, c, xi, G.bp_qle, gb.nb[q],
                                                             part + (size_t)5 * B * kGroupBlocks * q, s)));
                        sweep_edges += (unsigned long long)gp[q].edges();
                        HIPCHK((launch_pull_b<T, T, B>(t, ctl, gp[q], w, h, 0, s)));
                    }
                    HIPCHK(launch_decide_gs_b<B>(t, ctl, ngr, gb, part, sums, c, l1 ? 1 : 0, tol, pull_thr,
                                                 sweep_edges, s));
                    continue;
                }
                HIPCHK(launch_reserve_b<T, B>(t, ctl, nN, h, w, pibar, G.deg, G.rp_nn, c, xi, l1 ? 1 : 0, tol,
                                              pull_thr, force, (unsigned long long)pullp.edges(), part, s));
                if (force != 2) HIPCHK(launch_push_b<T, B>(t, ctl, G.bp_push_nn[slot], w, h, check_mode, s));
                if (force != 1) HIPCHK((launch_pull_b<T, T, B>(t, ctl, pullp, w, h, check_mode, s)));
            }
            HIPCHK(hipMemcpyAsync(hc, ctl, sizeof(CtlB), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hc->stop_after < t) {
                stopped = true;
                break;
            }
            double worst = 0.0;
            for (int j = 0; j < kb; ++j)
                if (hc->col_stop[j] >= t) worst = std::max(worst, hc->last_bound[j]);
            ordered = ordered_ok && hc->use_pull;  // dense frontier: ordered sweeps from here
            batch = next_batch(batch, bound_prev, worst, t - t_prev, tol, l1);
            if (ordered_ok && !ordered) batch = std::min(batch, 2);
            bound_prev = worst;
            t_prev = t;
        }
    } else {
        stopped = true;
    }
    if (nD > 0) HIPCHK(launch_phase2_b<T, B>(n, nN, G.perm, ss, h, pibar, G.deg, c, w2, xD, G.bp_pull_nd[slot], s));
    double *dst = out_dev ? pi_rows : outbuf;
    OutSet os;
    for (int j = 0; j < kMaxBatch; ++j) os.p[j] = j < kb ? dst + (size_t)j * n : nullptr;
    HIPCHK(launch_final_b<T, B>(ctl, n, nN, G.perm, kmask, os, h, pibar, xD, part, s));
    HIPCHK(hipEventRecord(ev_solve.b, s));
    HIPCHK(hipMemcpyAsync(hc, ctl, sizeof(CtlB), hipMemcpyDeviceToHost, s));
    if (!out_dev) HIPCHK(hipMemcpyAsync(pi_rows, outbuf, sizeof(double) * (size_t)kb * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st) {
        const double secs = elapsed_s(ev_solve.a, ev_solve.b);
        for (int j = 0; j < kb; ++j) {
            pr_stats z;
            memset(&z, 0, sizeof(z));
            z.sweeps = hc->col_sweeps[j];
            z.pull_sweeps = hc->pull_sweeps;
            z.edges_processed = (int64_t)hc->tot_edges[j] + G.mND;
            z.edges_traversed = (int64_t)hc->tot_traversed + G.mND;
            z.vertex_pushes = (int64_t)hc->tot_pushes[j];
            z.residual_l1 = hc->fin_sum[j] > 0 ? hc->fin_sn[j] / hc->fin_sum[j] : 0.0;
            z.l1_bound = hc->fin_sum[j] > 0 ? 2.0 * c / (1.0 - c) * hc->fin_sn[j] / hc->fin_sum[j] : 0.0;
            z.seconds_solve = secs;
            z.seconds_preprocess = G.seconds_split;
            st[j] = z;
        }
    }
    return stopped ? PR_OK : PR_ENOCONV;
}


pr_status tune_impl(Graph &G, const pr_opts &o, int32_t reps, pr_tune_report *rep) {
    const double t_start = (double)clock_now_ns() * 1e-9;
    if (reps <= 0) reps = 2;
    pr_tune_report r;
    memset(&r, 0, sizeof(r));
    double *out = nullptr;
    HIPCHK(hipMalloc((void **)&out, sizeof(double) * (size_t)G.n));
    struct Free {
        double *p;
        ~Free() { (void)hipFree(p); }
    } fr{out};
    pr_opts op = o;
    op.flags = (o.flags & ~(PR_OUT_DEVICE | PR_PROFILE | PR_JACOBI)) | PR_OUT_DEVICE;
    const bool can_order = G.grp.size() > 2 && !G.grp_pull.empty();
    const bool rows0 = G.group_rows;
    double best = INFINITY;
    int best_i = 0;
    // times the current schedule and records it as a candidate (ordered: 0 synchronous,
    // 1 ordered over whole-row group plans, 2 ordered over the rows each group reaches)
    auto candidate = [&](int32_t shift) -> pr_status {
        double ms = INFINITY;
        int32_t sweeps = 0;
        for (int32_t q = 0; q <= reps; ++q) {
            pr_stats st;
            pr_status ps = op.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, true, nullptr, -1, op, out, &st)
                                                      : solve_ifp_t<double>(G, true, nullptr, -1, op, out, &st);
            if (ps < 0) return ps;
            if (q > 0) ms = std::min(ms, st.seconds_solve * 1e3);
            sweeps = st.sweeps;
        }
        if (r.candidates >= PR_TUNE_MAX) return PR_OK;
        const int i = r.candidates++;
        r.tile_shift[i] = shift;
        r.groups[i] = G.prefer_ordered ? (int32_t)G.grp.size() - 1 : 1;
        r.ordered[i] = G.prefer_ordered ? (G.group_rows ? 2 : 1) : 0;
        r.ms[i] = ms;
        r.sweeps[i] = sweeps;
        if (ms < best) {
            best = ms;
            best_i = i;
        }
        return PR_OK;
    };
    for (int32_t shift = 2; shift <= 4; ++shift) {
        pr_status ps = replan(G, 1 << shift, G.stream);
        if (ps != PR_OK) return ps;
        for (int ord = 0; ord <= (can_order ? 1 : 0); ++ord) {
            G.prefer_ordered = ord == 1;
            ps = candidate(shift);
            if (ps != PR_OK) return ps;
        }
    }
    // at the tile size of the fastest ordered candidate: the other form of the group plans,
    // then other group counts in both forms (the best count grows with a sweep's work: more
    // groups pass more mass on within a sweep but add launches and row work)
    const int32_t k0 = can_order ? (int32_t)G.grp.size() - 1 : 1;
    int32_t k_built = k0;
    int best_ord = -1;
    for (int i = 0; i < r.candidates; ++i)
        if (r.ordered[i] != 0 && (best_ord < 0 || r.ms[i] < r.ms[best_ord])) best_ord = i;
    if (best_ord >= 0) {
        const int32_t shift = r.tile_shift[best_ord];
        pr_status ps = replan(G, 1 << shift, G.stream);
        if (ps != PR_OK) return ps;
        G.prefer_ordered = true;
        G.group_rows = !rows0;
        ps = candidate(shift);
        if (ps != PR_OK) return ps;
        for (int32_t k : {3, 4, 6, 8}) {
            if (k == k0) continue;
            ps = build_groups(G, k, G.stream);
            if (ps != PR_OK) return ps;
            k_built = k;
            if ((int32_t)G.grp.size() - 1 != k) continue;  // too few vertices for k groups
            for (int rows = 1; rows >= 0; --rows) {
                G.group_rows = rows == 1;
                ps = candidate(shift);
                if (ps != PR_OK) return ps;
            }
        }
    }
    r.chosen = best_i;
    pr_status ps = replan(G, 1 << r.tile_shift[best_i], G.stream);
    if (ps != PR_OK) return ps;
    const int32_t k_best = r.ordered[best_i] != 0 ? r.groups[best_i] : k0;
    if (k_best != k_built) {
        ps = build_groups(G, k_best, G.stream);
        if (ps != PR_OK) return ps;
    }
    G.prefer_ordered = r.ordered[best_i] != 0;
    G.group_rows = r.ordered[best_i] == 0 ? rows0 : r.ordered[best_i] == 2;
    // Batched solves under the chosen schedule: an ordered sweep of a batch gathers every
    // group over the rows it reaches for all columns, which costs more than one synchronous
    // gather, and single-source columns gain fewer sweeps from the ordering on some graphs
    // (the layered DAG) than on others; time a 16-source PPR batch both ways, keep the faster
    r.batch_ordered = -1;
    if (G.prefer_ordered && G.nN > 0 && G.nP == 0) {  // a peeled graph's PPR runs one source at a time
        int32_t srcs[kBatch];
        for (int j = 0; j < kBatch; ++j) {
            // the first non-dangling vertex at or after an evenly spaced original id
            int64_t v = (int64_t)((2 * j + 1) * (double)G.n / (2 * kBatch));
            for (int64_t k = 0; k < G.n && G.dangling(v); ++k) v = (v + 1) % G.n;
            srcs[j] = (int32_t)v;
        }
        // the batch's output: when the device cannot hold it, batches keep their default
        double *outb = nullptr;
        const bool room = hipMalloc((void **)&outb, sizeof(double) * kBatch * (size_t)G.n) == hipSuccess;
        if (!room) (void)hipGetLastError();
        Free fb{outb};
        double ms2[2] = {INFINITY, INFINITY};
        if (room) G.batch_order = 1;
        for (int form = 0; room && form < 2; ++form) {  // 0: ordered once dense, 1: synchronous
            pr_opts ob = op;
            if (form == 1) ob.flags |= PR_JACOBI;
            for (int32_t q = 0; q <= reps; ++q) {
                pr_stats st[kBatch];
                ps = op.residual == PR_RES_FP32 ? solve_ppr_batch_t<float, kBatch>(G, srcs, kBatch, ob, outb, st)
                                                : solve_ppr_batch_t<double, kBatch>(G, srcs, kBatch, ob, outb, st);
                if (ps < 0) return ps;
                if (q > 0) ms2[form] = std::min(ms2[form], st[0].seconds_solve * 1e3);
            }
        }
        if (room) {
            G.batch_order = ms2[0] <= ms2[1] ? 1 : 0;
            r.batch_ordered = G.batch_order;
            r.batch_ms[0] = ms2[0];
            r.batch_ms[1] = ms2[1];
        }
    }
    r.seconds = (double)clock_now_ns() * 1e-9 - t_start;
    if (rep) *rep = r;
    return PR_OK;
}

template pr_status solve_ifp_t<float>(const Graph &, bool, const double *, int32_t, const pr_opts &, double *,
                                      pr_stats *, const WarmArgs *, const ExtWorkspace *);
template pr_status solve_ifp_t<double>(const Graph &, bool, const double *, int32_t, const pr_opts &, double *,
                                       pr_stats *, const WarmArgs *, const ExtWorkspace *);
template size_t solve_ifp_bytes<float>(const Graph &, bool, const double *, const pr_opts &, bool);
template size_t solve_ifp_bytes<double>(const Graph &, bool, const double *, const pr_opts &, bool);
template pr_status solve_power_t<float>(const Graph &, const double *, const pr_opts &, double *, pr_stats *);
template pr_status solve_power_t<double>(const Graph &, const double *, const pr_opts &, double *, pr_stats *);
template pr_status solve_ppr_batch_t<float, 8>(const Graph &, const int32_t *, int, const pr_opts &, double *,
                                               pr_stats *);
template pr_status solve_ppr_batch_t<float, 16>(const Graph &, const int32_t *, int, const pr_opts &, double *,
                                                pr_stats *);
template pr_status solve_ppr_batch_t<double, 8>(const Graph &, const int32_t *, int, const pr_opts &, double *,
                                                pr_stats *);
template pr_status solve_ppr_batch_t<double, 16>(const Graph &, const int32_t *, int, const pr_opts &, double *,
                                                 pr_stats *);

}  // namespace host

pr_status batch_plans(Graph &G, int B, hipStream_t s) {
    return B == 8 ? host::ensure_batch_plans_impl<8>(G, s) : host::ensure_batch_plans_impl<16>(G, s);
}

}  // namespace prk
