// pr_host.hip -- host side of libpr.so: the C ABI of include/pr.h, graph
// upload and preparation, and the sweep loop of each solver.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/pr.h"
#include "../../include/pr_set.h"
#include "../../include/pr_warm.h"
#include "pr_internal.h"

using namespace prk;


namespace {

thread_local std::string g_err;

// per-sweep record of the calling thread's last PR_PROFILE solve
struct TraceRec {
    std::vector<int64_t> active, edges;
    std::vector<double> residual, bound;
    std::vector<int32_t> pulled;
};
thread_local TraceRec g_trace;

pr_status fail(pr_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

pr_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? PR_ENOMEM : PR_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

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

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t clock_now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

double elapsed_s(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

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
    if (flags & ~(PR_INPUT_DEVICE | PR_DEDUPE | PR_TILE_MASK | PR_GROUPS_MASK | PR_UNSORTED_IN | PR_PEEL))
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

    // Ordered sweeps (not for graph sets): source groups of equal N -> N out-edges in
    // the degree order, and for every epoch the in-lists of the N targets split by group.
    const int32_t ngroups_req = (flags & PR_GROUPS_MASK) ? (int32_t)((flags & PR_GROUPS_MASK) >> 12)
                                                         : (G.mNN >= ((int64_t)1 << 24) ? 4 : 1);
    if (!seg_of && G.nN > 0 && G.mNN > 0 && ngroups_req > 1) {
        std::vector<uint32_t> h_rpnn((size_t)G.nN + 1);
        HIPCHK(hipMemcpyAsync(h_rpnn.data(), G.rp_nn, sizeof(uint32_t) * ((size_t)G.nN + 1), hipMemcpyDeviceToHost,
                              s));
        HIPCHK(hipStreamSynchronize(s));
        G.grp.push_back(0);
        for (int32_t q = 1; q < ngroups_req; ++q) {
            const uint32_t target = (uint32_t)((double)G.mNN * q / ngroups_req);
            const int32_t b = (int32_t)(std::lower_bound(h_rpnn.begin(), h_rpnn.end(), target) - h_rpnn.begin());
            if (b > G.grp.back() && b < G.nN) G.grp.push_back(b);
        }
        G.grp.push_back(G.nN);
        uint32_t *d_gc;
        HIPCHK(tmp.alloc(&d_gc, (size_t)n + 1));
        for (size_t e = 0; e < G.epochs.size(); ++e) {
            std::vector<MPPlan> plans, plans_all;
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
                MPPlan pl, pla;
                HIPCHK(make_plan(pl, gp, gs, G.nN, ge[0]));
                HIPCHK(make_plan(pla, gp, gs, (int32_t)n, ge[1]));
                plans.push_back(pl);
                plans_all.push_back(pla);
            }
            G.grp_pull.push_back(plans);
            G.grp_pull_all.push_back(plans_all);
        }
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

// ---------------------------------------------------------------------------
// options / inputs
// ---------------------------------------------------------------------------
pr_status check_opts(const pr_opts &o, bool power) {
    if (!(o.c > 0.0 && o.c < 1.0)) return fail(PR_EINVAL, "c must be in (0, 1)");
    if (o.stop != PR_STOP_XI && o.stop != PR_STOP_L1) return fail(PR_EINVAL, "unknown stop rule");
    if (o.residual != PR_RES_FP64 && o.residual != PR_RES_FP32) return fail(PR_EINVAL, "unknown residual type");
    if (o.max_sweeps < 0) return fail(PR_EINVAL, "max_sweeps < 0");
    const uint32_t known =
        PR_P_DEVICE | PR_OUT_DEVICE | PR_IFP2_LITERAL | PR_FORCE_PUSH | PR_FORCE_PULL | PR_PROFILE | PR_JACOBI;
    if (o.flags & ~known) return fail(PR_EINVAL, "unknown option flag");
    if ((o.flags & PR_FORCE_PUSH) && (o.flags & PR_FORCE_PULL))
        return fail(PR_EINVAL, "PR_FORCE_PUSH and PR_FORCE_PULL together");
    if (power || o.stop == PR_STOP_L1) {
        if (!(o.l1_tol > 0.0) || !isfinite(o.l1_tol)) return fail(PR_EINVAL, "l1_tol must be > 0 and finite");
    }
    if (!power && o.stop == PR_STOP_XI) {
        if (!(o.xi > 0.0) || !isfinite(o.xi)) return fail(PR_EINVAL, "xi must be > 0 and finite");
    }
    return PR_OK;
}

// Solve workspace: one contiguous device allocation (cached on the graph) plus
// a pinned host copy of the control block.
struct Workspace {
    Graph *g = nullptr;
    char *base = nullptr;
    size_t bytes = 0;
    bool cached = false;
    Ctl *hctl = nullptr;  // pinned
    ~Workspace() {
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

pr_status acquire_ws(Graph &G, size_t bytes, Workspace &ws) {
    ws.g = &G;
    ws.bytes = bytes;
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
                    const double **p_used, double *pscale, hipStream_t s) {
    *p_used = nullptr;
    *pscale = 1.0;
    if (!p) return PR_OK;
    double sum = 0.0;
    if (o.flags & PR_P_DEVICE) {
        HIPCHK(hipMemsetAsync(sumbad, 0, 2 * sizeof(double), s));
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
            double need = log(tol / bound_now) / log(rate);
            int k = (int)ceil(need) + 1;
            return std::min(64, std::max(2, k));
        }
    }
    return std::min(64, prev_batch * 2);
}

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
constexpr int kGroupBlocks = 1024;
constexpr size_t kPartDoubles = (size_t)5 * kGroupBlocks * kMaxGroups + kRedBlocks;
static_assert(kPartDoubles >= (size_t)5 * kRedBlocks, "partials");

// state of a warm start (device, original ids): read at the start, written at the end
struct WarmArgs {
    double *pibar;
    double *h;
};

template <typename T>
pr_status solve_ifp_t(const Graph &G, bool ifp2, const double *p, int32_t source, const pr_opts &o, double *pi,
                      pr_stats *st, const WarmArgs *warm = nullptr) {
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

    size_t bytes = carve_size<T>(n) + carve_size<T>(nN) + carve_size<double>(nN) + carve_size<double>(nD) +
                   carve_size<double>(nN + G.nP) + carve_size<double>(out_dev ? 0 : n) + carve_size<Ctl>(1) +
                   carve_size<Trace>(1) + carve_size<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0) +
                   carve_size<double>(2) + carve_size<double>(kPartDoubles) +
                   (warm ? 2 * carve_size<double>(nN) + 3 * carve_size<double>(nD) : 0);
    Workspace ws;
    pr_status ps = acquire_ws(const_cast<Graph &>(G), bytes, ws);
    if (ps != PR_OK) return ps;
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

    InitArgs a{};
    a.n = n;
    a.nN = nN;
    a.perm = G.perm;
    a.source = source;
    a.uniform = (p == nullptr && source < 0);
    ps = prepare_p(G, p, o, pdev, sumbad, &a.p, &a.pscale, s);
    if (ps != PR_OK) return ps;

    EventPair ev_solve;
    SweepTimer timer;
    timer.on = o.flags & PR_PROFILE;
    HIPCHK(hipEventRecord(ev_solve.a, s));
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
    bool ordered = ordered_ok && a.uniform && !warm;
    GroupBlocks gb{};
    gb.stride = kGroupBlocks;
    for (int q = 0; q < ngr && q < kMaxGroups; ++q)
        gb.nb[q] = (int32_t)std::min<int64_t>(
            kGroupBlocks, std::max<int64_t>(1, ((int64_t)G.grp[q + 1] - G.grp[q] + 1023) / 1024));
    const double sT = (double)sizeof(T);
    int t = 0;
    bool stopped = false;
    if (nN > 0) {
        // a solve that may turn to ordered sweeps checks its frontier after two sweeps
        int batch = (ordered_ok && !ordered) ? 2 : (l1 ? 8 : 16);
        double bound_prev = -1.0;
        int t_prev = 0;
        while (t < max_sweeps) {
            int nb = std::min(batch, max_sweeps - t);
            for (int k = 0; k < nb; ++k, ++t) {
                const MPPlan &pullp = pull_plan(t);
                // a gather reads every live in-edge; scatter when the active edges are fewer than half of them
                const unsigned long long pull_edges = (unsigned long long)pullp.edges();
                const unsigned long long pull_thr = (unsigned long long)(0.5 * (double)pull_edges) + 1;
                if (ordered) {
                    size_t e = 0;
                    while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
                    unsigned long long sweep_edges = 0;
                    for (int q = 0; q < ngr; ++q) {
                        HIPCHK(launch_reserve_range<T>(t, ctl, G.grp[q], G.grp[q + 1], h, w, pibar, G.deg, G.rp_nn, c,
                                                       xi, ifp2 ? 1 : 0, gb.nb[q],
                                                       part + (size_t)5 * kGroupBlocks * q, s));
                        const MPPlan &pl = ifp2 ? G.grp_pull[e][q] : G.grp_pull_all[e][q];
                        sweep_edges += (unsigned long long)pl.edges();
                        const KernelEvents ev =
                            timer.next(t, 1, (double)pl.edges() * (4.0 + sT) + (double)pl.R * (4.0 + 2.0 * sT));
                        HIPCHK(launch_pull<T, T>(t, ctl, pl, w, h, 0, s, TileSkip(), ev));
                    }
                    HIPCHK(launch_decide_gs<T>(t, ctl, tr, nN, h, ngr, gb, part,
                                               part + (size_t)5 * kGroupBlocks * ngr, c, l1 ? 1 : 0, tol, pull_thr,
                                               sweep_edges, s));
                    continue;
                }
                HIPCHK(launch_reserve<T>(t, ctl, tr, nN, h, w, pibar, G.deg, G.rp_nn, c, xi, ifp2 ? 1 : 0, l1 ? 1 : 0,
                                         tol, pull_thr, force, pull_edges, part, s));
                if (force != 2) {
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
            ordered = ordered_ok && ws.hctl->use_pull;  // dense frontier: ordered sweeps from here
            batch = next_batch(batch, bound_prev, ws.hctl->last_bound, t - t_prev, tol, l1);
            bound_prev = ws.hctl->last_bound;
            t_prev = t;
        }
    } else {
        stopped = true;
    }
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
    double *dst = out_dev ? pi : outbuf;
    HIPCHK(launch_final_ifp<T>(ctl, a, h, pibar, xD, ifp2 ? 1 : 0, literal ? 1 : 0, dst, part, s));
    if (warm) HIPCHK(launch_warm_export<T>(n, nN, G.perm, h, pibar, hDn, warm->pibar, warm->h, s));
    HIPCHK(hipEventRecord(ev_solve.b, s));
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
        z.residual_l1 = r.fin_sum > 0 ? r.fin_sn / r.fin_sum : 0.0;
        const double k = literal ? 2.0 / (1.0 - c) : 2.0 * c / (1.0 - c);
        z.l1_bound = r.fin_sum > 0 ? k * r.fin_sn / r.fin_sum : 0.0;
        if (warm) {
            // signed residuals: unnormalised error E <= c / (1 - c) sum|h_N|, the exact mass is at
            // least fin_sum - E, and normalising costs (1 + sum|x| / sum x) E / (that mass)
            const double E = c / (1.0 - c) * r.fin_sn;
            const double den = r.fin_sum - E;
            z.l1_bound = den > 0 ? (1.0 + r.fin_abs / r.fin_sum) * E / den : INFINITY;
        }
        z.seconds_solve = elapsed_s(ev_solve.a, ev_solve.b);
        z.seconds_preprocess = ifp2 ? G.seconds_split : 0.0;
        if (timer.on) {
            std::vector<unsigned long long> trc((size_t)std::min(r.sweeps + 1, kMaxTrace));
            std::vector<unsigned long long> tre(trc.size());
            std::vector<double> trs(trc.size()), trb(trc.size());
            if (!trc.empty()) {
                HIPCHK(hipMemcpy(trc.data(), tr->cnt, sizeof(unsigned long long) * trc.size(), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(tre.data(), tr->edges, sizeof(unsigned long long) * tre.size(), hipMemcpyDeviceToHost));
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
    size_t bytes = carve_size<double>(n) * 2 + carve_size<WT>(nN) + carve_size<double>(out_dev ? 0 : n) +
                   carve_size<Ctl>(1) + carve_size<double>(p && !(o.flags & PR_P_DEVICE) ? n : 0) +
                   carve_size<double>(2) + carve_size<double>(5 * kRedBlocks);
    Workspace ws;
    pr_status ps = acquire_ws(const_cast<Graph &>(G), bytes, ws);
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
    HIPCHK(hipMemcpyAsync(ws.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (!out_dev) HIPCHK(hipMemcpyAsync(pi, outbuf, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Ctl &r = *ws.hctl;
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
    return stopped ? PR_OK : PR_ENOCONV;
}

// Plans for the batched kernels of width B (tiles of (kBlock / B) * kMPK items),
// built once per graph and width on the first batched solve.
template <int B>
pr_status ensure_batch_plans_impl(Graph &G, hipStream_t s) {
    constexpr int slot = B == 8 ? 0 : 1;
    std::lock_guard<std::mutex> lk(G.bp_mu);
    if (G.bp_ready[slot]) return PR_OK;
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
    return PR_OK;
}

// IFP2 for kb <= kBatch single-source PPR queries at once (pr_batch.hip):
// column-interleaved residuals, per-column management, one gather serving all
// columns.  pi_rows[r * n ...] receives the vector of srcs[r].
template <typename T, int B>
pr_status solve_ppr_batch_t(const Graph &Gc, const int32_t *srcs, int kb, const pr_opts &o, double *pi_rows,
                            pr_stats *st) {
    constexpr int slot = B == 8 ? 0 : 1;
    Graph &G = const_cast<Graph &>(Gc);
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

    size_t bytes = carve_size<T>((size_t)n * B) + carve_size<T>((size_t)nN * B) + carve_size<double>((size_t)nN * B) +
                   carve_size<double>((size_t)nD * B) + carve_size<double>((size_t)nN * B) +
                   carve_size<double>(out_dev ? 0 : (size_t)kb * n) + carve_size<CtlB>(1) +
                   carve_size<double>((size_t)4 * B * kRedBlocks);
    Workspace ws;
    ps = acquire_ws(G, bytes, ws);
    if (ps != PR_OK) return ps;
    Carve cv{ws.base};
    T *h = cv.take<T>((size_t)n * B);
    T *w = cv.take<T>((size_t)nN * B);
    double *pibar = cv.take<double>((size_t)nN * B);
    double *xD = cv.take<double>((size_t)nD * B);
    double *w2 = cv.take<double>((size_t)nN * B);
    double *outbuf = cv.take<double>(out_dev ? 0 : (size_t)kb * n);
    CtlB *ctl = cv.take<CtlB>(1);
    double *part = cv.take<double>((size_t)4 * B * kRedBlocks);
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

    const int force = (o.flags & PR_FORCE_PUSH) ? 1 : ((o.flags & PR_FORCE_PULL) ? 2 : 0);
    const int check_mode = force == 0;
    auto pull_plan = [&](int t) -> const MPPlan & {
        size_t e = 0;
        while (e + 1 < G.epochs.size() && G.epochs[e + 1].t_start <= t) ++e;
        return G.bp_pull_nn[slot][e];
    };
    int t = 0;
    bool stopped = false;
    if (nN > 0) {
        int batch = l1 ? 8 : 16;
        double bound_prev = -1.0;
        int t_prev = 0;
        while (t < max_sweeps) {
            const int nbt = std::min(batch, max_sweeps - t);
            for (int k = 0; k < nbt; ++k, ++t) {
                const MPPlan &pullp = pull_plan(t);
                // a gather serves every column; scatter when the active (vertex, column) edges are few
                const double pull_thr = 0.25 * (double)pullp.edges();
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
            batch = next_batch(batch, bound_prev, worst, t - t_prev, tol, l1);
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

// ---------------------------------------------------------------------------
// graph sets (include/pr_set.h)
// ---------------------------------------------------------------------------
}  // namespace

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
    std::vector<MPPlan> grp_pull;          // gather plan of each group's in-edges (owned by the union)
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

namespace {

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
    pr_status ps = acquire_ws(const_cast<Graph &>(G), bytes, ws);
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
                if (force != 2) HIPCHK(launch_push<T>(t, ctl, G.push_nn, w, h, force == 0, s, TileSkip{S.d_tg_push, gs}));
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

// Rebuild every single-vector merge-path plan of the graph for tiles of kBlock * tile_k
// items (the batched kernels keep their own plans).
pr_status replan(Graph &G, int32_t tile_k, hipStream_t s);
hipError_t replan_plan(Graph &G, MPPlan &p, int32_t tile_k, hipStream_t s);

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
// One plan of G (its split-point array owned by G) rebuilt for tiles of kBlock * tile_k items.
hipError_t replan_plan(Graph &G, MPPlan &p, int32_t tile_k, hipStream_t s) {
    const int32_t ipb = kBlock * tile_k;
    if (p.ipb == ipb) return hipSuccess;
    const int32_t blocks = (int32_t)(((int64_t)p.items + ipb - 1) / ipb);
    uint2 *np = nullptr;
    hipError_t e = hipMalloc((void **)&np, sizeof(uint2) * ((size_t)std::max(blocks, 0) + 1));
    if (e != hipSuccess) return e;
    auto it = std::find(G.allocs.begin(), G.allocs.end(), (void *)p.plan);
    if (it != G.allocs.end()) {
        G.allocs.erase(it);
        G.device_bytes -= (int64_t)sizeof(uint2) * ((int64_t)p.blocks + 1);
    }
    (void)hipFree(p.plan);
    G.allocs.push_back((void *)np);
    G.device_bytes += (int64_t)sizeof(uint2) * ((int64_t)blocks + 1);
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
    for (auto &p : G.lvl_pull) HIPCHK(one(p));
    HIPCHK(hipStreamSynchronize(s));
    G.tile_k = tile_k;
    return PR_OK;
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
    double best = INFINITY;
    int best_i = 0;
    for (int32_t shift = 2; shift <= 4; ++shift) {
        pr_status ps = replan(G, 1 << shift, G.stream);
        if (ps != PR_OK) return ps;
        for (int ord = 0; ord <= (can_order ? 1 : 0); ++ord) {
            G.prefer_ordered = ord == 1;
            double ms = INFINITY;
            int32_t sweeps = 0;
            for (int32_t q = 0; q <= reps; ++q) {
                pr_stats st;
                ps = op.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, true, nullptr, -1, op, out, &st)
                                                : solve_ifp_t<double>(G, true, nullptr, -1, op, out, &st);
                if (ps < 0) return ps;
                if (q > 0) ms = std::min(ms, st.seconds_solve * 1e3);
                sweeps = st.sweeps;
            }
            const int i = r.candidates++;
            r.tile_shift[i] = shift;
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
    pr_status ps = replan(G, 1 << r.tile_shift[best_i], G.stream);
    if (ps != PR_OK) return ps;
    G.prefer_ordered = r.ordered[best_i] == 1;
    r.seconds = (double)clock_now_ns() * 1e-9 - t_start;
    if (rep) *rep = r;
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

}  // namespace

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
pr_status set_error(pr_status st, const std::string &msg) { return fail(st, msg); }
pr_status batch_plans(Graph &G, int B, hipStream_t s) {
    return B == 8 ? ensure_batch_plans_impl<8>(G, s) : ensure_batch_plans_impl<16>(G, s);
}
void clear_error() { g_err.clear(); }
}  // namespace prk

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
    if (op.flags & (PR_FORCE_PUSH | PR_FORCE_PULL | PR_P_DEVICE))
        return fail(PR_EINVAL, "tuning times the automatic schedule of global solves");
    ps = enter(g);
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
    if (op.flags & (PR_FORCE_PUSH | PR_FORCE_PULL | PR_P_DEVICE | PR_IFP2_LITERAL | PR_PROFILE))
        return fail(PR_EINVAL, "tuning times the automatic schedule of set solves");
    ps = enter(s->u);
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
    if (op.flags & (PR_P_DEVICE | PR_IFP2_LITERAL | PR_PROFILE))
        return fail(PR_EINVAL, "option flag not supported for graph sets");
    ps = enter(s->u);
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
    pr_status worst = PR_OK;
    try {
        // groups of kBatch sources share one batched solve; a lone source runs alone, as
        // does every source on a peeled graph (the batched sweeps cover every non-dangling row)
        const int32_t width = G.nP > 0 ? 1 : kBatch;
        for (int32_t r = 0; r < k; r += width) {
            const int kb = (int)std::min<int32_t>(width, k - r);
            double *rows = pi + (size_t)r * (size_t)G.n;
            pr_stats *sr = st ? st + r : nullptr;
            pr_status rs;
            if (kb == 1) {
                rs = op.residual == PR_RES_FP32 ? solve_ifp_t<float>(G, true, nullptr, sources[r], op, rows, sr)
                                                : solve_ifp_t<double>(G, true, nullptr, sources[r], op, rows, sr);
            } else if (kb <= 8) {
                rs = op.residual == PR_RES_FP32 ? solve_ppr_batch_t<float, 8>(G, sources + r, kb, op, rows, sr)
                                                : solve_ppr_batch_t<double, 8>(G, sources + r, kb, op, rows, sr);
            } else {
                rs = op.residual == PR_RES_FP32 ? solve_ppr_batch_t<float, 16>(G, sources + r, kb, op, rows, sr)
                                                : solve_ppr_batch_t<double, 16>(G, sources + r, kb, op, rows, sr);
            }
            if (rs < 0) return rs;
            if (rs > worst) worst = rs;
        }
    } catch (const std::bad_alloc &) {
        return fail(PR_ENOMEM, "host allocation");
    }
    return worst;
}

}  // extern "C"
