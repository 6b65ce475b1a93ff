// pr_set_host.hip -- host side of graph sets (include/pr_set.h): the union upload,
// per-graph vertex groups of ordered sweeps, the set solve loop and its autotuner.
#include "pr_host.h"

namespace prk {
namespace host {


// Vertex groups of ordered sweeps for a graph set: within every graph the rule of one
// graph (boundaries at equal shares of its N -> N out-edges in the degree order; a
// boundary that does not advance leaves an empty group), and per group the in-edges of
// all non-dangling rows whose source is in the group, with their gather plan.
pr_status set_groups(pr_graph_set &S, int32_t ngr) {
    Graph &G = S.u->g;
    hipStream_t s = G.stream;
    const int32_t nN = G.nN, k = S.k;
    std::vector<uint32_t> rp((size_t)nN + 1);
    HIPCHK(hipMemcpy(rp.data(), G.rp_nn, sizeof(uint32_t) * ((size_t)nN + 1), hipMemcpyDeviceToHost));
    std::vector<uint8_t> gid((size_t)nN);
    std::vector<std::vector<int32_t>> goff((size_t)ngr, std::vector<int32_t>((size_t)k + 1, 0));
    std::vector<std::vector<int32_t>> gbase((size_t)ngr, std::vector<int32_t>((size_t)k, 0));
    std::vector<int32_t> b((size_t)ngr + 1);
    for (int32_t g = 0; g < k; ++g) {
        const int32_t a = S.offN[(size_t)g], nNg = S.offN[(size_t)g + 1] - a;
        const uint32_t e0 = rp[(size_t)a], mg = rp[(size_t)(a + nNg)] - e0;
        b[0] = 0;
        for (int32_t q = 1; q < ngr; ++q) {
            const uint32_t target = e0 + (uint32_t)((double)mg * q / ngr);
            const int32_t x = (int32_t)(std::lower_bound(rp.begin() + a, rp.begin() + a + nNg + 1, target) -
                                        (rp.begin() + a));
            b[(size_t)q] = std::min(std::max(x, b[(size_t)q - 1]), nNg);
        }
        b[(size_t)ngr] = nNg;
        for (int32_t q = 0; q < ngr; ++q) {
            const int32_t len = b[(size_t)q + 1] - b[(size_t)q];
            for (int32_t j = b[(size_t)q]; j < b[(size_t)q + 1]; ++j) gid[(size_t)(a + j)] = (uint8_t)q;
            gbase[(size_t)q][(size_t)g] = a + b[(size_t)q] - goff[(size_t)q][(size_t)g];
            goff[(size_t)q][(size_t)g + 1] = goff[(size_t)q][(size_t)g] + len;
        }
    }
    DevBufs tmp;
    uint8_t *d_gid;
    uint32_t *d_cnt, *d_scan;
    HIPCHK(tmp.alloc(&d_gid, (size_t)nN));
    HIPCHK(tmp.alloc(&d_cnt, (size_t)nN + 1));
    HIPCHK(tmp.alloc(&d_scan, scan_tmp_elems((int64_t)nN + 1)));
    HIPCHK(hipMemcpy(d_gid, gid.data(), (size_t)nN, hipMemcpyHostToDevice));
    auto galloc = [&](auto **p, size_t count) -> hipError_t {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc((void **)p, bytes);
        if (e == hipSuccess) {
            G.allocs.push_back((void *)*p);
            G.device_bytes += (int64_t)bytes;
        }
        return e;
    };
    S.ngr = ngr;
    for (int32_t q = 0; q < ngr; ++q) {
        int32_t *d_off = nullptr, *d_base = nullptr;
        HIPCHK(hipMalloc((void **)&d_off, sizeof(int32_t) * ((size_t)k + 1)));
        S.d_goff.push_back(d_off);
        HIPCHK(hipMalloc((void **)&d_base, sizeof(int32_t) * (size_t)k));
        S.d_gbase.push_back(d_base);
        HIPCHK(hipMemcpy(d_off, goff[(size_t)q].data(), sizeof(int32_t) * ((size_t)k + 1), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_base, gbase[(size_t)q].data(), sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice));
        S.glen.push_back(goff[(size_t)q][(size_t)k]);
        // the group's in-edges of every non-dangling row (full lists: no depth epochs)
        uint32_t *gp;
        int32_t *gsrc;
        HIPCHK(galloc(&gp, (size_t)nN + 1));
        HIPCHK(launch_live_count(nN, G.in_ptr, G.in_src, G.depth, 0, 0, INT_MAX, d_cnt, s, d_gid, q));
        HIPCHK(launch_scan_u32(d_cnt, gp, nN, d_scan, s));
        uint32_t ge = 0;
        HIPCHK(hipMemcpyAsync(&ge, gp + nN, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(galloc(&gsrc, (size_t)ge));
        HIPCHK(launch_live_fill(nN, G.in_ptr, G.in_src, G.depth, 0, 0, INT_MAX, gp, gsrc, s, d_gid, q));
        MPPlan pl;
        pl.rp = gp;
        pl.idx = gsrc;
        pl.R = nN;
        pl.items = (uint32_t)((int64_t)nN + ge);
        pl.ipb = kBlock * G.tile_k;
        HIPCHK(galloc(&pl.plan, (size_t)(((int64_t)pl.items + pl.ipb - 1) / pl.ipb) + 1));
        HIPCHK(launch_plan(pl, s));
        S.grp_pull.push_back(pl);
        uint2 *tg = nullptr;
        HIPCHK(hipMalloc((void **)&tg, sizeof(uint2) * (size_t)std::max<int32_t>(pl.blocks, 1)));
        S.d_tg_grp.push_back(tg);
        HIPCHK(launch_set_tile_graphs(pl, S.d_offN, k, tg, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return PR_OK;
}

pr_status set_upload_impl(int32_t k, const int64_t *n, const int64_t *const *row_ptr, const int32_t *const *col,
                          uint32_t flags, pr_graph_set **out) {
    if (!out) return fail(PR_EINVAL, "out is NULL");
    if (k < 1) return fail(PR_EINVAL, "k must be >= 1");
    if (!n || !row_ptr || !col) return fail(PR_EINVAL, "NULL array");
    if (flags & ~(PR_TILE_MASK | PR_GROUPS_MASK)) return fail(PR_EINVAL, "unknown upload flag for a graph set");
    std::unique_ptr<pr_graph_set> S(new pr_graph_set());
    S->k = k;
    S->n_g.assign(n, n + k);
    S->off.assign((size_t)k + 1, 0);
    int64_t mt = 0;
    for (int32_t g = 0; g < k; ++g) {
        if (n[g] < 1) return fail(PR_EINVAL, "every graph needs n >= 1");
        const int64_t *rp = row_ptr[g];
        if (!rp) return fail(PR_EINVAL, "row_ptr entry is NULL");
        if (rp[0] != 0) return fail(PR_EINVAL, "row_ptr[0] != 0");
        for (int64_t i = 0; i < n[g]; ++i)
            if (rp[i + 1] < rp[i]) return fail(PR_EINVAL, "row_ptr is not non-decreasing");
        const int64_t mg = rp[n[g]];
        if (mg > 0 && !col[g]) return fail(PR_EINVAL, "col entry is NULL");
        for (int64_t e = 0; e < mg; ++e)
            if (col[g][e] < 0 || col[g][e] >= n[g]) return fail(PR_EINVAL, "col entry out of [0, n)");
        S->off[(size_t)g + 1] = S->off[(size_t)g] + n[g];
        mt += mg;
        if (S->off[(size_t)g + 1] >= ((int64_t)1 << 31) || mt >= ((int64_t)1 << 31))
            return fail(PR_EINVAL, "set exceeds 2^31 vertices or edges");
    }
    const int64_t nt = S->off[(size_t)k];
    std::vector<int64_t> urp((size_t)nt + 1);
    std::vector<int32_t> ucol((size_t)std::max<int64_t>(mt, 1));
    std::vector<int32_t> seg((size_t)nt);
    S->offN.assign((size_t)k + 1, 0);
    S->offD.assign((size_t)k + 1, 0);
    S->mND_g.assign((size_t)k, 0);
    S->m_g.assign((size_t)k, 0);
    int64_t e_at = 0;
    for (int32_t g = 0; g < k; ++g) {
        const int64_t *rp = row_ptr[g];
        const int64_t o = S->off[(size_t)g];
        int32_t nd = 0;
        for (int64_t i = 0; i < n[g]; ++i) {
            urp[(size_t)(o + i)] = e_at + rp[i];
            seg[(size_t)(o + i)] = g;
            nd += rp[i + 1] == rp[i];
        }
        int64_t mnd = 0;
        for (int64_t e = 0; e < rp[n[g]]; ++e) {
            const int32_t v = col[g][e];
            ucol[(size_t)(e_at + e)] = (int32_t)(o + v);
            mnd += rp[v + 1] == rp[v];
        }
        S->mND_g[(size_t)g] = mnd;
        S->m_g[(size_t)g] = rp[n[g]];
        S->offN[(size_t)g + 1] = S->offN[(size_t)g] + (int32_t)(n[g] - nd);
        S->offD[(size_t)g + 1] = S->offD[(size_t)g] + nd;
        e_at += rp[n[g]];
    }
    urp[(size_t)nt] = e_at;
    pr_status ps = upload_impl(nt, mt, urp.data(), ucol.data(), flags & PR_TILE_MASK, seg.data(), &S->u);
    if (ps != PR_OK) return ps;
    const Graph &G = S->u->g;
    if (G.nN != S->offN[(size_t)k]) return fail(PR_EDEVICE, "internal: region sizes of the set disagree");
    HIPCHK(hipMalloc((void **)&S->d_offN, sizeof(int32_t) * ((size_t)k + 1)));
    HIPCHK(hipMalloc((void **)&S->d_offD, sizeof(int32_t) * ((size_t)k + 1)));
    HIPCHK(hipMemcpy(S->d_offN, S->offN.data(), sizeof(int32_t) * ((size_t)k + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_offD, S->offD.data(), sizeof(int32_t) * ((size_t)k + 1), hipMemcpyHostToDevice));
    auto tile_graphs = [&](const MPPlan &p, uint2 **dst) -> hipError_t {
        hipError_t e = hipMalloc((void **)dst, sizeof(uint2) * (size_t)std::max<int32_t>(p.blocks, 1));
        if (e != hipSuccess) return e;
        return launch_set_tile_graphs(p, S->d_offN, k, *dst, G.stream);
    };
    HIPCHK(tile_graphs(G.push_nn, &S->d_tg_push));
    S->d_tg_pull.assign(G.epochs.size(), nullptr);
    for (size_t e = 0; e < G.epochs.size(); ++e) HIPCHK(tile_graphs(G.epochs[e].pull_nn, &S->d_tg_pull[e]));
    HIPCHK(hipStreamSynchronize(G.stream));
    const int32_t ngr = (flags & PR_GROUPS_MASK) ? (int32_t)((flags & PR_GROUPS_MASK) >> 12) : 4;
    if (ngr > 1 && G.nN > 0 && G.mNN > 0) {
        ps = set_groups(*S, ngr);
        if (ps != PR_OK) return ps;
    }
    *out = S.release();
    return PR_OK;
}

template <typename T>
pr_status solve_set_t(const pr_graph_set &S, const double *cg, const pr_opts &o, double *pi, pr_stats *st) {
    const Graph &G = S.u->g;
    hipStream_t s = o.stream ? (hipStream_t)o.stream : G.stream;
    const int64_t n = G.n;
    const int32_t nN = G.nN, nD = G.nD, k = S.k;
    const bool out_dev = o.flags & PR_OUT_DEVICE;
    const bool l1 = o.stop == PR_STOP_L1;
    const double tol = l1 ? o.l1_tol * (1.0 - 1e-6) : 0.0;
    const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 100000;
    const int force = (o.flags & PR_FORCE_PUSH) ? 1 : ((o.flags & PR_FORCE_PULL) ? 2 : 0);

    std::vector<SetG> hs((size_t)k);
    for (int32_t g = 0; g < k; ++g) {
        SetG &x = hs[(size_t)g];
        memset(&x, 0, sizeof(x));
        const double c = cg ? cg[g] : o.c;
        if (!(c > 0.0 && c < 1.0)) return fail(PR_EINVAL, "every c must be in (0, 1)");
        const int32_t nNg = S.offN[(size_t)g + 1] - S.offN[(size_t)g];
        x.c = c;
        // as for one graph: the threshold at which an empty frontier certifies the bound
        x.xi = l1 ? o.l1_tol * (1.0 - c) / (2.0 * c) * (double)S.n_g[(size_t)g] / (double)std::max<int32_t>(nNg, 1) *
                        (1.0 - 1e-9)
                  : o.xi;
        x.sx = (double)S.n_g[(size_t)g];
        x.m_nn = (double)(S.m_g[(size_t)g] - S.mND_g[(size_t)g]);
        x.last_bound = INFINITY;
        x.stop_after = nNg > 0 ? INT_MAX : -1;
    }

    size_t bytes = carve_size<T>(n) + carve_size<T>(nN) + carve_size<double>(nN) + carve_size<double>(nD) +
                   carve_size<double>(nN) + carve_size<double>(out_dev ? 0 : n) + carve_size<Ctl>(1) +
                   carve_size<SetG>((size_t)k);
    Workspace ws;
    pr_status ps = acquire_ws(const_cast<Graph &>(G), bytes, ws, s);
    if (ps != PR_OK) return ps;
    Carve cv{ws.base};
    T *h = cv.take<T>(n);
    T *w = cv.take<T>(nN);
    double *pibar = cv.take<double>(nN);
    double *xD = cv.take<double>(nD);
    double *w2 = cv.take<double>(nN);
    double *outbuf = cv.take<double>(out_dev ? 0 : n);
    Ctl *ctl = cv.take<Ctl>(1);
    SetG *gs = cv.take<SetG>((size_t)k);

    EventPair ev_solve;
    HIPCHK(hipEventRecord(ev_solve.a, s));
    Ctl hc;
    memset(&hc, 0, sizeof(hc));
    hc.stop_after = INT_MAX;
    HIPCHK(hipMemcpyAsync(ctl, &hc, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(gs, hs.data(), sizeof(SetG) * (size_t)k, hipMemcpyHostToDevice, s));
    HIPCHK(launch_set_init<T>(n, nN, h, pibar, s));

    int t = 0;
    bool stopped = nN == 0;
    // ordered sweeps over the vertex groups while the frontier is dense (every vertex
    // starts active), as for one graph
    const bool ordered_ok = S.ngr > 1 && S.prefer_ordered && force == 0 && !(o.flags & PR_JACOBI);
    bool ordered = ordered_ok;
    if (nN > 0) {
        int batch = l1 ? 8 : 16;
        double bound_prev = -1.0;
        int t_prev = 0;
        while (t < max_sweeps) {
            const int nb = std::min(batch, max_sweeps - t);
            for (int q = 0; q < nb; ++q, ++t) {
                if (ordered) {
                    for (int32_t r = 0; r < S.ngr; ++r) {
                        HIPCHK(launch_set_reserve<T>(t, ctl, gs, S.d_goff[(size_t)r], S.d_gbase[(size_t)r], k,
                                                     S.glen[(size_t)r], h, w, pibar, G.deg, G.rp_nn, s));
                        HIPCHK(launch_pull<T, T>(t, ctl, S.grp_pull[(size_t)r], w, h, 0, s,
                                                 TileSkip{S.d_tg_grp[(size_t)r], gs}));
                    }
                    HIPCHK(launch_set_sum_h<T>(t, ctl, gs, S.d_offN, k, nN, h, s));
                    HIPCHK(launch_set_decide(t, ctl, gs, k, l1 ? 1 : 0, tol, 1.0, force, 1, s));
                    continue;
                }
                size_t e = 0;
                while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
                const MPPlan &pullp = G.epochs[e].pull_nn;
                // share of the N -> N edges still in this epoch's gather lists
                const double live_frac = G.mNN > 0 ? (double)pullp.edges() / (double)G.mNN : 0.0;
                HIPCHK(launch_set_reserve<T>(t, ctl, gs, S.d_offN, nullptr, k, nN, h, w, pibar, G.deg, G.rp_nn, s));
                HIPCHK(launch_set_decide(t, ctl, gs, k, l1 ? 1 : 0, tol, live_frac, force, 0, s));
                if (force != 2)
                    HIPCHK(launch_push<T>(t, ctl, G.push_nn, w, h, force == 0, s, TileSkip{S.d_tg_push, gs}));
                if (force != 1)
                    HIPCHK(launch_pull<T, T>(t, ctl, pullp, w, h, force == 0, s, TileSkip{S.d_tg_pull[e], gs}));
            }
            HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (ws.hctl->stop_after < t) {
                stopped = true;
                break;
            }
            ordered = ordered_ok && ws.hctl->use_pull;  // a thin frontier scatters instead
            batch = next_batch(batch, bound_prev, ws.hctl->last_bound, t - t_prev, tol, l1);
            bound_prev = ws.hctl->last_bound;
            t_prev = t;
        }
    }
    if (nD > 0) {
        HIPCHK(launch_set_phase2_prep<T>(n, nN, gs, S.d_offN, k, h, pibar, G.deg, w2, xD, s));
        HIPCHK(launch_pull<double, double>(-1, ctl, G.pull_nd, w2, xD, 0, s));
    }
    double *dst = out_dev ? pi : outbuf;
    HIPCHK(launch_set_final<T>(n, nN, gs, S.d_offN, S.d_offD, k, G.perm, h, pibar, xD, dst, s));
    HIPCHK(hipEventRecord(ev_solve.b, s));
    HIPCHK(hipMemcpyAsync(hs.data(), gs, sizeof(SetG) * (size_t)k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (!out_dev) HIPCHK(hipMemcpyAsync(pi, outbuf, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double secs = elapsed_s(ev_solve.a, ev_solve.b);
    bool all = true;
    for (int32_t g = 0; g < k; ++g) {
        const SetG &x = hs[(size_t)g];
        const bool conv = x.stop_after < INT_MAX || stopped;
        all = all && conv;
        if (!st) continue;
        pr_stats z;
        memset(&z, 0, sizeof(z));
        z.sweeps = x.sweeps;
        z.pull_sweeps = ws.hctl->pull_sweeps;
        z.edges_processed = (int64_t)x.tot_edges + S.mND_g[(size_t)g];
        z.edges_traversed = z.edges_processed;
        z.vertex_pushes = (int64_t)x.tot_pushes;
        z.residual_l1 = x.fin_sum > 0 ? x.fin_sn / x.fin_sum : 0.0;
        z.l1_bound = x.fin_sum > 0 ? 2.0 * x.c / (1.0 - x.c) * x.fin_sn / x.fin_sum : 0.0;
        z.seconds_solve = secs;
        z.seconds_preprocess = G.seconds_split;
        st[g] = z;
    }
    return all ? PR_OK : PR_ENOCONV;
}

// A graph set's plans for a new tile size, with the tile-to-graph tables that follow them.
pr_status set_replan(pr_graph_set &S, int32_t tile_k) {
    Graph &G = S.u->g;
    hipStream_t s = G.stream;
    pr_status ps = replan(G, tile_k, s);
    if (ps != PR_OK) return ps;
    for (MPPlan &p : S.grp_pull) HIPCHK(replan_plan(G, p, tile_k, s));
    auto retable = [&](const MPPlan &p, uint2 *&dst) -> hipError_t {
        if (dst) (void)hipFree(dst);
        dst = nullptr;
        hipError_t e = hipMalloc((void **)&dst, sizeof(uint2) * (size_t)std::max<int32_t>(p.blocks, 1));
        if (e != hipSuccess) return e;
        return launch_set_tile_graphs(p, S.d_offN, S.k, dst, s);
    };
    HIPCHK(retable(G.push_nn, S.d_tg_push));
    for (size_t e = 0; e < G.epochs.size(); ++e) HIPCHK(retable(G.epochs[e].pull_nn, S.d_tg_pull[e]));
    for (size_t q = 0; q < S.grp_pull.size(); ++q) HIPCHK(retable(S.grp_pull[q], S.d_tg_grp[q]));
    HIPCHK(hipStreamSynchronize(s));
    return PR_OK;
}

// The autotuner of one graph (tune_impl) for a graph set: every tile size with
// synchronous and, when the set has vertex groups, ordered sweeps; the set keeps the
// fastest schedule.
pr_status set_tune_impl(pr_graph_set &S, const double *cg, const pr_opts &o, int32_t reps, pr_tune_report *rep) {
    Graph &G = S.u->g;
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
    op.flags = (o.flags & ~(PR_OUT_DEVICE | PR_JACOBI)) | PR_OUT_DEVICE;
    std::vector<pr_stats> st((size_t)S.k);
    const bool can_order = S.ngr > 1;
    double best = INFINITY;
    int best_i = 0;
    for (int32_t shift = 2; shift <= 4; ++shift) {
        pr_status ps = set_replan(S, 1 << shift);
        if (ps != PR_OK) return ps;
        for (int ord = 0; ord <= (can_order ? 1 : 0); ++ord) {
            S.prefer_ordered = ord == 1;
            double ms = INFINITY;
            int32_t sweeps = 0;
            for (int32_t q = 0; q <= reps; ++q) {
                ps = op.residual == PR_RES_FP32 ? solve_set_t<float>(S, cg, op, out, st.data())
                                                : solve_set_t<double>(S, cg, op, out, st.data());
                if (ps < 0) return ps;
                if (q > 0) ms = std::min(ms, st[0].seconds_solve * 1e3);
                sweeps = 0;
                for (const pr_stats &x : st) sweeps = std::max(sweeps, x.sweeps);
            }
            const int i = r.candidates++;
            r.tile_shift[i] = shift;
            r.groups[i] = ord ? S.ngr : 1;
            r.ordered[i] = ord;
            r.ms[i] = ms;
            r.sweeps[i] = sweeps;
            if (ms < best) {
                best = ms;
                best_i = i;
            }
        }
    }
    r.chosen = best_i;
    pr_status ps = set_replan(S, 1 << r.tile_shift[best_i]);
    if (ps != PR_OK) return ps;
    S.prefer_ordered = r.ordered[best_i] == 1;
    r.seconds = (double)clock_now_ns() * 1e-9 - t_start;
    if (rep) *rep = r;
    return PR_OK;
}

template pr_status solve_set_t<float>(const pr_graph_set &, const double *, const pr_opts &, double *, pr_stats *);
template pr_status solve_set_t<double>(const pr_graph_set &, const double *, const pr_opts &, double *, pr_stats *);

}  // namespace host
}  // namespace prk
