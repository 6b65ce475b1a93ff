// pr_upload.hip -- graph upload of libpr.so: validation, weak-dangling levels,
// the device vertex order, the split CSR of IFP2, in-edge lists, merge-path plans,
// unreferenced-depth epochs and the vertex groups of ordered sweeps.
#include "pr_host.h"

namespace prk {
namespace host {

// ---------------------------------------------------------------------------
// graph upload
// ---------------------------------------------------------------------------

// Levels of weakly dangling vertices (PR_PEEL): lev = 0 for a dangling vertex, L >= 1 for
// one whose out-edges all lead to vertices of levels below L, -1 for the core.  Rounds of
// deletion from the dangling vertices along reversed edges: each vertex counts down its
// out-edges into vertices not yet peeled and peels in the round that takes the last one.
// Returns the number of levels.
int32_t peel_levels(int64_t n, const int64_t *rp, const int32_t *col, std::vector<int32_t> &lev) {
    const int64_t m = rp[n];
    std::vector<int64_t> ip((size_t)n + 1, 0);
    for (int64_t e = 0; e < m; ++e) ip[(size_t)col[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) ip[(size_t)i + 1] += ip[(size_t)i];
    std::vector<int32_t> isrc((size_t)std::max<int64_t>(m, 1));
    {
        std::vector<int64_t> cur(ip.begin(), ip.end() - 1);
        for (int64_t v = 0; v < n; ++v)
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) isrc[(size_t)cur[(size_t)col[e]]++] = (int32_t)v;
    }
    std::vector<int32_t> rem((size_t)n), front, next;
    lev.assign((size_t)n, -1);
    for (int64_t v = 0; v < n; ++v) {
        rem[(size_t)v] = (int32_t)(rp[v + 1] - rp[v]);
        if (rem[(size_t)v] == 0) {
            lev[(size_t)v] = 0;
            front.push_back((int32_t)v);
        }
    }
    int32_t levels = 0;
    for (int32_t L = 1; L <= PR_PEEL_MAX_LEVELS && !front.empty(); ++L) {
        next.clear();
        for (int32_t v : front)
            for (int64_t e = ip[(size_t)v]; e < ip[(size_t)v + 1]; ++e) {
                const int32_t u = isrc[(size_t)e];
                if (--rem[(size_t)u] == 0) {
                    lev[(size_t)u] = L;
                    next.push_back(u);
                }
            }
        if (!next.empty()) levels = L;
        front.swap(next);
    }
    return levels;
}

// Device vertex order: non-dangling vertices first, by decreasing out-degree
// (ties by original id), then dangling vertices in original order.  A vertex's
// out-degree is how often its weight is gathered by a pull sweep (and, on
// these graphs, tracks how often it is a scatter target), so the most-read
// entries of the residual-sized vectors share cache lines and stay resident in
// the per-XCD L2.  Stable LSD radix sort on the complemented degree.  With a
// segment index per vertex (a graph set: segments are contiguous id ranges)
// the order is by segment first, so every segment's non-dangling vertices,
// and its dangling ones, stay contiguous.  With peel levels (lev, see peel_levels) the
// sorted prefix is the core, followed by the peeled vertices by level from the highest
// down (original order within a level); lvl_lo receives the first new id of each level,
// then of the dangling vertices, then n.
int32_t degree_order(int64_t n, const int64_t *rp, const int32_t *seg_of, const int32_t *lev, int32_t levels,
                     std::vector<int32_t> &perm, std::vector<int32_t> &newid, std::vector<int32_t> &lvl_lo) {
    std::vector<int32_t> nd;
    std::vector<uint32_t> key;
    nd.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        if (lev ? lev[i] < 0 : rp[i + 1] > rp[i]) nd.push_back((int32_t)i);
    const size_t nN = nd.size();
    std::vector<int32_t> tmp(nN);
    std::vector<uint32_t> cnt(1u << 16);
    for (int pass = 0; pass < (seg_of ? 4 : 2); ++pass) {
        const int sh = 16 * (pass & 1);
        std::fill(cnt.begin(), cnt.end(), 0u);
        auto kf = [&](int32_t v) {
            const uint32_t key = pass < 2 ? ~(uint32_t)(rp[v + 1] - rp[v]) : (uint32_t)seg_of[v];
            return (key >> sh) & 0xffffu;
        };
        for (int32_t v : nd) cnt[kf(v)]++;
        uint32_t run = 0;
        for (auto &c : cnt) {
            uint32_t x = c;
            c = run;
            run += x;
        }
        for (int32_t v : nd) tmp[cnt[kf(v)]++] = v;
        nd.swap(tmp);
    }
    perm.resize((size_t)n);
    newid.resize((size_t)n);
    size_t k = 0;
    for (int32_t v : nd) perm[k++] = v;
    lvl_lo.clear();
    if (lev) {
        std::vector<size_t> pos((size_t)levels + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            if (lev[i] > 0) pos[(size_t)lev[i]]++;
        for (int32_t L = levels; L >= 1; --L) {  // highest level first
            const size_t c = pos[(size_t)L];
            pos[(size_t)L] = k;
            lvl_lo.push_back((int32_t)k);
            k += c;
        }
        for (int64_t i = 0; i < n; ++i)
            if (lev[i] > 0) perm[pos[(size_t)lev[i]]++] = (int32_t)i;
        lvl_lo.push_back((int32_t)k);
        lvl_lo.push_back((int32_t)n);
    }
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] == rp[i]) perm[k++] = (int32_t)i;
    for (int64_t j = 0; j < n; ++j) newid[perm[j]] = (int32_t)j;
    return (int32_t)nN;
}

pr_status upload_impl(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                      const int32_t *seg_of, pr_graph **out) {
    if (!out) return fail(PR_EINVAL, "out is NULL");
    if (flags & ~(PR_INPUT_DEVICE | PR_DEDUPE | PR_TILE_MASK | PR_GROUPS_MASK | PR_UNSORTED_IN | PR_PEEL |
                  PR_GROUP_ALL_ROWS))
        return fail(PR_EINVAL, "unknown upload flag");
    if ((flags & PR_PEEL) && seg_of) return fail(PR_EINVAL, "graph sets are not peeled");
    const uint32_t tile_shift = (flags & PR_TILE_MASK) >> 8;
    if (tile_shift != 0 && (tile_shift < 2 || tile_shift > 4)) return fail(PR_EINVAL, "tile shift must be 2, 3 or 4");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(PR_EINVAL, "n must be in [1, 2^31)");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PR_EINVAL, "m must be in [0, 2^31)");
    if (!row_ptr) return fail(PR_EINVAL, "row_ptr is NULL");
    if (m > 0 && !col) return fail(PR_EINVAL, "col is NULL");
    const bool dev_in = flags & PR_INPUT_DEVICE;

    // row_ptr is validated on the host (host inputs are checked before any HIP call)
    std::vector<int64_t> hrp;
    const int64_t *rp = row_ptr;
    if (dev_in) {
        hrp.resize((size_t)n + 1);
        HIPCHK(hipMemcpy(hrp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
        rp = hrp.data();
    }
    if (rp[0] != 0) return fail(PR_EINVAL, "row_ptr[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(PR_EINVAL, "row_ptr is not non-decreasing");
    if (rp[n] != m) return fail(PR_EINVAL, "row_ptr[n] != m");

    // optional de-duplication (host): sort every row and drop repeats
    std::vector<int64_t> drp;
    std::vector<int32_t> dcol;
    const int32_t *hcol = dev_in ? nullptr : col;
    if (flags & PR_DEDUPE) {
        std::vector<int32_t> tmp;
        if (dev_in) {
            tmp.resize((size_t)std::max<int64_t>(m, 1));
            if (m) HIPCHK(hipMemcpy(tmp.data(), col, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
            hcol = tmp.data();
        }
        for (int64_t e = 0; e < m; ++e)
            if (hcol[e] < 0 || hcol[e] >= n) return fail(PR_EINVAL, "col entry out of [0, n)");
        drp.assign((size_t)n + 1, 0);
        dcol.reserve((size_t)m);
        for (int64_t i = 0; i < n; ++i) {
            size_t b = dcol.size();
            dcol.insert(dcol.end(), hcol + rp[i], hcol + rp[i + 1]);
            std::sort(dcol.begin() + b, dcol.end());
            dcol.erase(std::unique(dcol.begin() + b, dcol.end()), dcol.end());
            drp[i + 1] = (int64_t)dcol.size();
        }
        m = (int64_t)dcol.size();
        rp = drp.data();
        hcol = dcol.data();
    }
    const bool col_on_device = dev_in && !(flags & PR_DEDUPE);
    int device = 0;
    HIPCHK(hipGetDevice(&device));

    std::unique_ptr<pr_graph> hg(new (std::nothrow) pr_graph());
    if (!hg) return fail(PR_ENOMEM, "host allocation");
    Graph &G = hg->g;
    G.n = n;
    G.m = m;
    G.device = device;
    G.tile_k = tile_shift ? (1 << tile_shift) : kMPK;
    HIPCHK(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
    hipStream_t s = G.stream;
    struct StreamGuard {
        Graph *g;
        bool keep = false;
        ~StreamGuard() {
            if (!keep) {
                for (void *p : g->allocs) (void)hipFree(p);
                g->allocs.clear();
                if (g->stream) (void)hipStreamDestroy(g->stream);
            }
        }
    } guard{&G};

    EventPair ev_all, ev_split;
    HIPCHK(hipEventRecord(ev_all.a, s));

    DevBufs tmp;
    int64_t *d_rp64;
    int32_t *d_col;
    HIPCHK(tmp.alloc(&d_rp64, (size_t)n + 1));
    HIPCHK(tmp.alloc(&d_col, (size_t)m));
    HIPCHK(hipMemcpyAsync(d_rp64, rp, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    if (m) {
        if (col_on_device) HIPCHK(hipMemcpyAsync(d_col, col, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
        else HIPCHK(hipMemcpyAsync(d_col, hcol, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    }
    // column range check before anything indexes with col
    unsigned int *d_bad;
    HIPCHK(tmp.alloc(&d_bad, 1));
    HIPCHK(hipMemsetAsync(d_bad, 0, sizeof(unsigned int), s));
    HIPCHK(launch_check_cols(d_col, m, n, d_bad, s));
    unsigned int h_bad = 0;
    HIPCHK(hipMemcpyAsync(&h_bad, d_bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h_bad) return fail(PR_EINVAL, "col entry out of [0, n)");

    auto galloc = [&](auto **p, size_t count) -> hipError_t {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc((void **)p, bytes);
        if (e == hipSuccess) {
            G.allocs.push_back((void *)*p);
            G.device_bytes += (int64_t)bytes;
        }
        return e;
    };

    // weakly dangling levels (PR_PEEL) need the columns on the host
    std::vector<int32_t> lev, ccol;
    int32_t levels = 0;
    if (flags & PR_PEEL) {
        const int32_t *pc = hcol;
        if (!pc) {
            ccol.resize((size_t)std::max<int64_t>(m, 1));
            if (m) HIPCHK(hipMemcpyAsync(ccol.data(), d_col, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            pc = ccol.data();
        }
        levels = peel_levels(n, rp, pc, lev);
        std::vector<int32_t>().swap(ccol);
    }

    // class of every vertex: swept (non-dangling; with PR_PEEL the core) or deferred
    uint32_t *d_isN, *d_scan;
    HIPCHK(tmp.alloc(&d_isN, (size_t)n));
    HIPCHK(tmp.alloc(&d_scan, scan_tmp_elems(std::max<int64_t>(n, m) + 1)));
    if (flags & PR_PEEL) {
        std::vector<uint32_t> is_core((size_t)n);
        for (int64_t i = 0; i < n; ++i) is_core[(size_t)i] = lev[(size_t)i] < 0 ? 1u : 0u;
        HIPCHK(hipMemcpyAsync(d_isN, is_core.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        HIPCHK(launch_degree_class(d_rp64, n, d_isN, s));
    }

    // vertex order on the device (see degree_order)
    std::vector<int32_t> h_perm, h_newid;
    G.nN = degree_order(n, rp, seg_of, lev.empty() ? nullptr : lev.data(), levels, h_perm, h_newid, G.lvl_lo);
    G.nD = (int32_t)(n - G.nN);
    G.nP = lev.empty() ? 0 : G.lvl_lo[(size_t)levels] - G.nN;
    const int32_t nNP = G.nN + G.nP;  // rows with out-edges
    std::vector<int32_t>().swap(lev);
    G.dangling_bits.assign((size_t)(n + 63) / 64, 0);
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] == rp[i]) G.dangling_bits[(size_t)i >> 6] |= 1ull << (i & 63);
    HIPCHK(galloc(&G.perm, (size_t)n));
    HIPCHK(galloc(&G.newid, (size_t)n));
    HIPCHK(hipMemcpyAsync(G.perm, h_perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(G.newid, h_newid.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));

    uint32_t *d_indeg_old, *d_indeg, *d_cnn, *d_cnd, *d_cursor;
    HIPCHK(tmp.alloc(&d_indeg_old, (size_t)n));
    HIPCHK(tmp.alloc(&d_indeg, (size_t)n));
    HIPCHK(hipMemsetAsync(d_indeg_old, 0, sizeof(uint32_t) * n, s));
    HIPCHK(launch_indegree(d_col, m, d_indeg_old, s));

    HIPCHK(tmp.alloc(&d_cnn, (size_t)nNP + 1));
    HIPCHK(tmp.alloc(&d_cnd, (size_t)nNP + 1));
    HIPCHK(galloc(&G.deg, (size_t)nNP));
    HIPCHK(galloc(&G.rp_nn, (size_t)nNP + 1));
    HIPCHK(galloc(&G.rp_nd, (size_t)nNP + 1));
    HIPCHK(hipEventRecord(ev_split.a, s));
    HIPCHK(launch_count_nn(d_rp64, d_col, d_isN, G.perm, nNP, d_cnn, d_cnd, G.deg, s));
    HIPCHK(launch_scan_u32(d_cnn, G.rp_nn, nNP, d_scan, s));
    HIPCHK(launch_scan_u32(d_cnd, G.rp_nd, nNP, d_scan, s));
    // edges of the swept rows into swept / deferred targets, and of all rows
    uint32_t h_mm[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(&h_mm[0], G.rp_nn + G.nN, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&h_mm[1], G.rp_nd + G.nN, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&h_mm[2], G.rp_nn + nNP, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&h_mm[3], G.rp_nd + nNP, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    G.mNN = h_mm[2];
    G.mND = h_mm[3];
    const int64_t mND_swept = h_mm[1];
    // a peeled vertex has no edge into the core
    if (h_mm[0] != h_mm[2] || G.mNN + G.mND != m) return fail(PR_EDEVICE, "internal: split edge count mismatch");
    HIPCHK(galloc(&G.col_nn, (size_t)G.mNN));
    HIPCHK(galloc(&G.col_nd, (size_t)G.mND));
    HIPCHK(launch_split_rows(d_rp64, d_col, d_isN, G.newid, G.perm, nNP, G.rp_nn, G.col_nn, G.rp_nd, G.col_nd, s));
    HIPCHK(hipEventRecord(ev_split.b, s));

    // in-edge lists (N targets first, then D targets)
    HIPCHK(launch_permute_u32(d_indeg_old, G.perm, n, d_indeg, s));
    HIPCHK(galloc(&G.in_ptr, (size_t)n + 1));
    HIPCHK(galloc(&G.in_src, (size_t)m));
    HIPCHK(launch_scan_u32(d_indeg, G.in_ptr, n, d_scan, s));
    HIPCHK(tmp.alloc(&d_cursor, (size_t)n));
    HIPCHK(hipMemcpyAsync(d_cursor, G.in_ptr, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_fill_csc(G.rp_nn, G.col_nn, nNP, d_cursor, G.in_src, s));
    HIPCHK(launch_fill_csc(G.rp_nd, G.col_nd, nNP, d_cursor, G.in_src, s));
    if (!(flags & PR_UNSORTED_IN)) HIPCHK(sort_in_lists(n, m, G.in_ptr, G.in_src, s));
    unsigned long long *d_zero;
    HIPCHK(tmp.alloc(&d_zero, 1));
    HIPCHK(hipMemsetAsync(d_zero, 0, sizeof(unsigned long long), s));
    HIPCHK(launch_count_zero(d_indeg, n, d_zero, s));

    // merge-path plans
    auto make_plan = [&](MPPlan &p, const uint32_t *rpp, const int32_t *idx, int32_t R, int64_t edges) -> hipError_t {
        p.rp = rpp;
        p.idx = idx;
        p.R = R;
        p.items = (uint32_t)(R + edges);
        p.ipb = kBlock * G.tile_k;
        int32_t blocks = (int32_t)(((int64_t)p.items + p.ipb - 1) / p.ipb);
        hipError_t e = galloc(&p.plan, (size_t)blocks + 1);
        if (e != hipSuccess) return e;
        if (R == 0) {
            p.blocks = 0;
            return hipSuccess;
        }
        return launch_plan(p, s);
    };
    HIPCHK(make_plan(G.push_nn, G.rp_nn, G.col_nn, G.nN, G.mNN));
    HIPCHK(make_plan(G.push_nd, G.rp_nd, G.col_nd, G.nN, mND_swept));
    HIPCHK(make_plan(G.pull_all, G.in_ptr, G.in_src, (int32_t)n, m));
    HIPCHK(make_plan(G.pull_nn, G.in_ptr, G.in_src, G.nN, G.mNN));
    HIPCHK(make_plan(G.pull_nd, G.in_ptr + G.nN, G.in_src, G.nD, G.mND));
    if (!G.lvl_lo.empty()) {  // PR_PEEL: one gather per deferred block
        std::vector<uint32_t> ip_lo(G.lvl_lo.size());
        for (size_t b = 0; b < G.lvl_lo.size(); ++b)
            HIPCHK(hipMemcpyAsync(&ip_lo[b], G.in_ptr + G.lvl_lo[b], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        G.lvl_pull.resize(G.lvl_lo.size() - 1);
        for (size_t b = 0; b + 1 < G.lvl_lo.size(); ++b)
            HIPCHK(make_plan(G.lvl_pull[b], G.in_ptr + G.lvl_lo[b], G.in_src, G.lvl_lo[b + 1] - G.lvl_lo[b],
                             (int64_t)ip_lo[b + 1] - ip_lo[b]));
    }
    {
        Epoch e0;
        e0.t_start = 0;
        e0.in_ptr = G.in_ptr;
        e0.in_src = G.in_src;
        e0.edges_all = m;
        e0.edges_nn = G.mNN;
        e0.pull_all = G.pull_all;
        e0.pull_nn = G.pull_nn;
        G.epochs.push_back(e0);
    }

    // Unreferenced depth of every non-dangling vertex (Kahn rounds over the N -> N
    // edges), then compacted in-edge lists for the sweeps after which whole depth
    // classes of sources can no longer push (section 3.3.3: unreferenced and weakly
    // unreferenced vertices leave the computation).
    HIPCHK(galloc(&G.depth, (size_t)nNP));
    if (G.nP > 0) {  // peeled sources never lose their in-edges from the compacted lists
        std::vector<int32_t> inf((size_t)G.nP, kDepthInf);
        HIPCHK(hipMemcpyAsync(G.depth + G.nN, inf.data(), sizeof(int32_t) * G.nP, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (G.nN > 0) {
        uint32_t *d_rem, *d_qc;
        int32_t *d_q0, *d_q1;
        HIPCHK(tmp.alloc(&d_rem, (size_t)G.nN));
        HIPCHK(tmp.alloc(&d_q0, (size_t)G.nN));
        HIPCHK(tmp.alloc(&d_q1, (size_t)G.nN));
        HIPCHK(tmp.alloc(&d_qc, 2));
        HIPCHK(hipMemsetAsync(d_qc, 0, 2 * sizeof(uint32_t), s));
        HIPCHK(launch_depth_init(G.nN, G.in_ptr, d_rem, G.depth, d_q0, d_qc, s));
        uint32_t qsize = 0;
        HIPCHK(hipMemcpyAsync(&qsize, d_qc, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int32_t round = 0;
        while (qsize > 0) {
            G.max_depth = round;
            HIPCHK(hipMemsetAsync(d_qc + 1, 0, sizeof(uint32_t), s));
            HIPCHK(launch_depth_step(d_q0, qsize, G.rp_nn, G.col_nn, d_rem, G.depth, round, d_q1, d_qc + 1, s));
            HIPCHK(hipMemcpyAsync(&qsize, d_qc + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            std::swap(d_q0, d_q1);
            ++round;
        }
        // live edges L(t) = sum of out-degrees of sources with depth >= t
        std::vector<int32_t> h_depth((size_t)G.nN);
        HIPCHK(hipMemcpy(h_depth.data(), G.depth, sizeof(int32_t) * G.nN, hipMemcpyDeviceToHost));
        const int32_t dmax = std::max<int32_t>(G.max_depth, 0);
        std::vector<int64_t> hist((size_t)dmax + 2, 0);  // [0..dmax] finite, [dmax+1] infinite
        for (int32_t k = 0; k < G.nN; ++k) {
            const int32_t v = h_perm[k];
            const int64_t dg = rp[v + 1] - rp[v];
            const int32_t d = h_depth[k];
            hist[d == kDepthInf ? (size_t)dmax + 1 : (size_t)d] += dg;
        }
        std::vector<int64_t> live((size_t)dmax + 3, 0);  // live[t] = sum_{d >= t} hist[d]
        for (int32_t t = dmax + 1; t >= 0; --t) live[(size_t)t] = live[(size_t)t + 1] + hist[(size_t)t];
        std::vector<int32_t> starts;
        int64_t cur = m;
        for (int32_t t = 1; t <= dmax + 1 && (int)starts.size() + 1 < kMaxEpochs; ++t) {
            if ((double)live[(size_t)t] <= 0.97 * (double)cur) {
                starts.push_back(t);
                cur = live[(size_t)t];
            }
        }
        uint32_t *d_cnt;
        HIPCHK(tmp.alloc(&d_cnt, (size_t)n + 1));
        for (int32_t t0 : starts) {
            Epoch ep;
            ep.t_start = t0;
            HIPCHK(galloc(&ep.in_ptr, (size_t)n + 1));
            HIPCHK(launch_live_count((int32_t)n, G.in_ptr, G.in_src, G.depth, t0, 0, INT_MAX, d_cnt, s));
            HIPCHK(launch_scan_u32(d_cnt, ep.in_ptr, n, d_scan, s));
            uint32_t h_e[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(&h_e[0], ep.in_ptr + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&h_e[1], ep.in_ptr + G.nN, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ep.edges_all = h_e[0];
            ep.edges_nn = h_e[1];
            HIPCHK(galloc(&ep.in_src, (size_t)ep.edges_all));
            HIPCHK(launch_live_fill((int32_t)n, G.in_ptr, G.in_src, G.depth, t0, 0, INT_MAX, ep.in_ptr, ep.in_src,
                                    s));
            HIPCHK(make_plan(ep.pull_all, ep.in_ptr, ep.in_src, (int32_t)n, ep.edges_all));
            HIPCHK(make_plan(ep.pull_nn, ep.in_ptr, ep.in_src, G.nN, ep.edges_nn));
            G.epochs.push_back(ep);
        }
    }

    // Ordered sweeps (not for graph sets): vertex groups and their gather plans
    const int32_t ngroups_req = (flags & PR_GROUPS_MASK) ? (int32_t)((flags & PR_GROUPS_MASK) >> 12)
                                                         : (G.mNN >= ((int64_t)1 << 24) ? 4 : 1);
    G.group_rows = !(flags & PR_GROUP_ALL_ROWS);
    if (!seg_of) {
        pr_status gs = build_groups(G, ngroups_req, s);
        if (gs != PR_OK) return gs;
    }

    unsigned long long h_zero = 0;
    HIPCHK(hipMemcpyAsync(&h_zero, d_zero, sizeof(h_zero), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(ev_all.b, s));
    HIPCHK(hipStreamSynchronize(s));
    G.n_unref = (int64_t)h_zero;
    G.seconds_upload = elapsed_s(ev_all.a, ev_all.b);
    G.seconds_split = elapsed_s(ev_split.a, ev_split.b);
    guard.keep = true;
    *out = hg.release();
    return PR_OK;
}


// Vertex groups of ordered sweeps: the non-dangling vertices split into k groups of equal
// N -> N out-edge counts in the degree order, and for every depth epoch the in-lists of the
// targets split by group, both as whole-row gather plans and as plans over only the rows
// each group reaches.  Replaces the groups the graph had (their memory is freed; k <= 1
// leaves none); the plans take the graph's current tile size.
pr_status build_groups(Graph &G, int32_t k, hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    ++G.grp_version;  // weights derived from the old groups are stale from here
    for (void *p : G.grp_allocs) (void)hipFree(p);
    G.grp_allocs.clear();
    G.device_bytes -= G.grp_bytes;
    G.grp_bytes = 0;
    G.grp.clear();
    G.grp_pull.clear();
    G.grp_pull_all.clear();
    G.grp_pull_rows.clear();
    G.grp_pull_all_rows.clear();
    for (int b = 0; b < 2; ++b) G.bp_grp[b].clear();  // built for the batched kernels from the groups
    G.bp_qle = nullptr;
    const int64_t n = G.n;
    if (k <= 1 || G.nN == 0 || G.mNN == 0) return PR_OK;
    // a failed build leaves no groups (the graph then sweeps synchronously)
    struct Undo {
        Graph &G;
        bool keep = false;
        ~Undo() {
            if (keep) return;
            G.grp.clear();
            G.grp_pull.clear();
            G.grp_pull_all.clear();
            G.grp_pull_rows.clear();
            G.grp_pull_all_rows.clear();
        }
    } undo{G};
    auto galloc = [&](auto **p, size_t count) -> hipError_t {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        *p = nullptr;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = hipMalloc((void **)p, bytes);
        if (e == hipSuccess) {
            G.grp_allocs.push_back((void *)*p);
            G.grp_bytes += (int64_t)bytes;
            G.device_bytes += (int64_t)bytes;
        }
        return e;
    };
    auto make_plan = [&](MPPlan &p, const uint32_t *rpp, const int32_t *idx, int32_t R, int64_t edges) -> hipError_t {
        p.rp = rpp;
        p.idx = idx;
        p.R = R;
        p.items = (uint32_t)(R + edges);
        p.ipb = kBlock * G.tile_k;
        const int32_t blocks = (int32_t)(((int64_t)p.items + p.ipb - 1) / p.ipb);
        hipError_t e = galloc(&p.plan, (size_t)blocks + 1);
        if (e != hipSuccess) return e;
        if (R == 0) {
            p.blocks = 0;
            return hipSuccess;
        }
        return launch_plan(p, s);
    };
    DevBufs tmp;
    uint32_t *d_scan;
    HIPCHK(tmp.alloc(&d_scan, scan_tmp_elems(n + 1)));
    std::vector<uint32_t> h_rpnn((size_t)G.nN + 1);
    HIPCHK(hipMemcpyAsync(h_rpnn.data(), G.rp_nn, sizeof(uint32_t) * ((size_t)G.nN + 1), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    G.grp.push_back(0);
    for (int32_t q = 1; q < k; ++q) {
        const uint32_t target = (uint32_t)((double)G.mNN * q / k);
        const int32_t b = (int32_t)(std::lower_bound(h_rpnn.begin(), h_rpnn.end(), target) - h_rpnn.begin());
        if (b > G.grp.back() && b < G.nN) G.grp.push_back(b);
    }
    G.grp.push_back(G.nN);
    uint32_t *d_gc, *d_flag, *d_pos;
    HIPCHK(tmp.alloc(&d_gc, (size_t)n + 1));
    HIPCHK(tmp.alloc(&d_flag, (size_t)n + 1));
    HIPCHK(tmp.alloc(&d_pos, (size_t)n + 1));
    // A group's gather over only the rows with an edge from the group (about 60 % of the
    // non-dangling rows each on R-MAT, 70 % on the layered DAG): rid names their targets
    // and rp their edges in the group's in-lists (off: the offsets over all R rows).
    auto make_group_plan = [&](MPPlan &p, const uint32_t *off, const int32_t *idx, int32_t R,
                               int64_t edges) -> hipError_t {
        hipError_t e = launch_row_flags(R, d_gc, d_flag, s);
        if (e == hipSuccess) e = launch_scan_u32(d_flag, d_pos, R, d_scan, s);
        uint32_t kept = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&kept, d_pos + R, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        int32_t *rid = nullptr;
        uint32_t *rpc = nullptr;
        e = galloc(&rid, (size_t)kept);
        if (e == hipSuccess) e = galloc(&rpc, (size_t)kept + 1);
        if (e == hipSuccess) e = launch_row_fill(R, d_gc, d_pos, off, rid, rpc, s);
        if (e == hipSuccess) e = make_plan(p, rpc, idx, (int32_t)kept, edges);
        p.rid = rid;
        return e;
    };
    for (size_t e = 0; e < G.epochs.size(); ++e) {
        std::vector<MPPlan> plans, plans_all, plans_rows, plans_all_rows;
        for (size_t q = 0; q + 1 < G.grp.size(); ++q) {
            uint32_t *gp;
            int32_t *gs;
            HIPCHK(galloc(&gp, (size_t)n + 1));
            HIPCHK(launch_live_count((int32_t)n, G.in_ptr, G.in_src, G.depth, G.epochs[e].t_start, G.grp[q],
                                     G.grp[q + 1], d_gc, s));
            HIPCHK(launch_scan_u32(d_gc, gp, n, d_scan, s));
            uint32_t ge[2] = {0, 0};  // edges into the non-dangling rows, into all rows
            HIPCHK(hipMemcpyAsync(&ge[0], gp + G.nN, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&ge[1], gp + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            HIPCHK(galloc(&gs, (size_t)ge[1]));
            HIPCHK(launch_live_fill((int32_t)n, G.in_ptr, G.in_src, G.depth, G.epochs[e].t_start, G.grp[q],
                                    G.grp[q + 1], gp, gs, s));
            MPPlan pl, pla, plr, plar;
            HIPCHK(make_plan(pl, gp, gs, G.nN, ge[0]));
            HIPCHK(make_plan(pla, gp, gs, (int32_t)n, ge[1]));
            HIPCHK(make_group_plan(plr, gp, gs, G.nN, ge[0]));
            HIPCHK(make_group_plan(plar, gp, gs, (int32_t)n, ge[1]));
            plans.push_back(pl);
            plans_all.push_back(pla);
            plans_rows.push_back(plr);
            plans_all_rows.push_back(plar);
        }
        G.grp_pull.push_back(plans);
        G.grp_pull_all.push_back(plans_all);
        G.grp_pull_rows.push_back(plans_rows);
        G.grp_pull_all_rows.push_back(plans_all_rows);
    }
    undo.keep = true;
    return PR_OK;
}

hipError_t replan_plan(Graph &G, MPPlan &p, int32_t tile_k, hipStream_t s) {
    const int32_t ipb = kBlock * tile_k;
    if (p.ipb == ipb) return hipSuccess;
    const int32_t blocks = (int32_t)(((int64_t)p.items + ipb - 1) / ipb);
    uint2 *np = nullptr;
    hipError_t e = hipMalloc((void **)&np, sizeof(uint2) * ((size_t)std::max(blocks, 0) + 1));
    if (e != hipSuccess) return e;
    // the plan array belongs to the graph's own list or to its vertex groups' list
    std::vector<void *> *owner = &G.allocs;
    auto it = std::find(G.allocs.begin(), G.allocs.end(), (void *)p.plan);
    if (it == G.allocs.end()) {
        auto jt = std::find(G.grp_allocs.begin(), G.grp_allocs.end(), (void *)p.plan);
        if (jt != G.grp_allocs.end()) {
            owner = &G.grp_allocs;
            it = jt;
        }
    }
    const bool grp = owner == &G.grp_allocs;
    if (it != owner->end()) {
        owner->erase(it);
        G.device_bytes -= (int64_t)sizeof(uint2) * ((int64_t)p.blocks + 1);
        if (grp) G.grp_bytes -= (int64_t)sizeof(uint2) * ((int64_t)p.blocks + 1);
    }
    (void)hipFree(p.plan);
    owner->push_back((void *)np);
    G.device_bytes += (int64_t)sizeof(uint2) * ((int64_t)blocks + 1);
    if (grp) G.grp_bytes += (int64_t)sizeof(uint2) * ((int64_t)blocks + 1);
    p.plan = np;
    p.ipb = ipb;
    if (p.R == 0) {
        p.blocks = 0;
        return hipSuccess;
    }
    return launch_plan(p, s);
}

pr_status replan(Graph &G, int32_t tile_k, hipStream_t s) {
    auto one = [&](MPPlan &p) -> hipError_t { return replan_plan(G, p, tile_k, s); };
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(one(G.push_nn));
    HIPCHK(one(G.push_nd));
    HIPCHK(one(G.pull_all));
    HIPCHK(one(G.pull_nn));
    HIPCHK(one(G.pull_nd));
    for (size_t e = 0; e < G.epochs.size(); ++e) {
        if (e == 0) {  // epoch 0 aliases the full lists
            G.epochs[0].pull_all = G.pull_all;
            G.epochs[0].pull_nn = G.pull_nn;
        } else {
            HIPCHK(one(G.epochs[e].pull_all));
            HIPCHK(one(G.epochs[e].pull_nn));
        }
    }
    for (auto &v : G.grp_pull)
        for (auto &p : v) HIPCHK(one(p));
    for (auto &v : G.grp_pull_all)
        for (auto &p : v) HIPCHK(one(p));
    for (auto &v : G.grp_pull_rows)
        for (auto &p : v) HIPCHK(one(p));
    for (auto &v : G.grp_pull_all_rows)
        for (auto &p : v) HIPCHK(one(p));
    for (auto &p : G.lvl_pull) HIPCHK(one(p));
    HIPCHK(hipStreamSynchronize(s));
    G.tile_k = tile_k;
    return PR_OK;
}

}  // namespace host
}  // namespace prk
