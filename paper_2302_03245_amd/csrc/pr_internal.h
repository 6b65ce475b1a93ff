// pr_internal.h -- device data layout and kernel launchers shared by the HIP
// translation units of libpr.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pr.h"

#include <mutex>
#include <string>
#include <vector>

namespace prk {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kMaxTrace = 4096;   // per-sweep trace entries kept on the device
constexpr int kRedBlocks = 1024;  // max workgroups of a streaming kernel that feeds a reduction
constexpr int kMaxGroups = 15;    // vertex groups of ordered sweeps
constexpr int kGroupBlocks = 1024;  // max workgroups of one group's reserve in an ordered sweep
// A single-vector or graph-set sweep scatters (one FP32 / FP64 atomic per active
// edge, about 21 G/s for random targets) while its active edges are below this
// share of the edges a gather would read (a gather reads all of them at about 200 G/s).
constexpr double kScatterShare = 0.1;
// A batched sweep scatters while its active (vertex, column) edges summed over the
// columns are below this share of the edges its gather would read (the gather
// serves all columns at once; the scatter's atomics of one edge hit adjacent columns).
constexpr double kScatterShareBatch = 0.25;
// A single-vector sweep scatters from a compacted frontier list (returning atomics, no
// pass over every vertex) while its active edges are below this share of a gather's.
constexpr double kListShare = 0.02;

// workgroups of each group's reserve in an ordered sweep; group g's five partial
// arrays (nb[g] entries each) start at part + 5 * stride * g
struct GroupBlocks {
    int32_t stride;
    int32_t nb[kMaxGroups];
};
// the vertex groups of ordered sweeps as id ranges: group q ends before end[q]
struct GroupEnds {
    int32_t ng;
    int32_t end[kMaxGroups];
};
// Partial sums of a batched solve of width B with ngr vertex groups (doubles): a
// synchronous sweep's reserve writes 4 rows of B columns, one entry per workgroup; an
// ordered sweep's group q writes 5 rows at 5 * B * kGroupBlocks * q; the ordered
// sweep's per-group row sums follow all of them.
inline size_t batch_part_doubles(int B, int ngr) {
    const size_t rows = (size_t)4 * B * kRedBlocks, grp = (size_t)5 * B * kGroupBlocks * ngr;
    return (rows > grp ? rows : grp) + (size_t)5 * B * ngr;
}
constexpr int32_t kDepthInf = 0x7fffffff;  // unreferenced depth of vertices on or below a cycle
constexpr int kMaxEpochs = 8;     // compacted in-edge lists kept per graph
constexpr int kMPK = 8;           // default merge-path items (rows + edges) per thread (4, 8 or 16)
constexpr int kBatch = 16;        // vectors per batched launch (a batch of <= 8 uses width 8)

// Merge-path work split over a CSR-like segment: rows r in [0, R) with edges
// [rp[r], rp[r+1]).  The item sequence lists the edges of a row followed by an
// end-of-row marker; item positions are diagonals of the merge of row ends
// with edge indices.  plan[b] = (row, edge) at diagonal b * items_per_block.
struct MPPlan {
    const uint32_t *rp = nullptr;  // device, R + 1 absolute edge offsets
    const int32_t *idx = nullptr;  // device, edge endpoint array (absolute offsets index it)
    int32_t R = 0;
    uint32_t items = 0;            // R + number of edges
    int32_t blocks = 0;
    int32_t ipb = 0;               // items per tile (kBlock x items per thread)
    uint2 *plan = nullptr;         // device, blocks + 1 entries (owned by the graph)
    const int32_t *rid = nullptr;  // device, R target-row ids when the plan keeps only the rows
                                   // with an edge in it (a vertex group's gather); null: rows 0 .. R-1
    int64_t edges() const { return (int64_t)items - R; }
};

// Control block of one solve (device memory).  Per-sweep accumulators are
// filled with atomics by every workgroup and consumed and reset by the last one.
struct alignas(128) Ctl {
    int32_t stop_after;   // sweeps with index > stop_after do nothing
    int32_t sweeps;       // sweeps that moved mass
    int32_t use_pull;     // mode of the current sweep's scatter/gather
    int32_t pull_sweeps;
    uint32_t bdone;       // last-block counters
    uint32_t fdone;
    int32_t signed_res;   // residuals may be negative (a warm start): the bound uses the signed form
    uint32_t pad0;
    double acc[4];        // per-sweep FP64 accumulators
    unsigned long long acc_cnt, acc_edges;
    double sx;            // running total mass sum(pibar + h) (+ untouched dangling mass for IFP2)
    double last_bound;    // bound certified at the last reserve
    unsigned long long tot_pushes, tot_edges, tot_traversed;
    // power method
    double pw_b;          // jump weight c * d^T x + (1 - c) * e^T x of the current iterate
    double pw_diff;       // ||x_t - x_{t-1}||_1 of the last iterate
    // finalisation
    double fin_sum, fin_sn;
    double fin_abs;       // sum |x| (equals fin_sum unless residuals went negative)
    double fin_res;       // sum |h| over the non-dangling vertices (fin_sn is weighted when the bound is)
    // a-posteriori check (PR_VERIFY): ||P'' pi - pi||_1, its rounding bound, sum(pi)
    double ver_r, ver_err, ver_sum;
    double ver_rf;        // sum_j f_j |r_j| with f_j the absorbing mass weight of row j (see launch_verify)
    double ver_beta;      // the second scale of the weighted bound (0: none)
    double ver_rf2;       // sum_j f_j |r_j| at that scale (infinite without one)
    // list sweeps (compacted frontier): entries of the two frontier lists and of the
    // lane / wave work lists of the scatter, indexed by sweep parity
    uint32_t fcnt[2], lcnt[2], wcnt[2], pad2[2];
    unsigned long long fedges[2];   // valid out-edges of the vertices in each frontier list
    unsigned long long last_edges;  // valid out-edges of the last decided sweep's active vertices
    double sn_last;                 // residual left on the non-dangling vertices after that sweep
};

// Per-vertex weights of the stop rule's error bound for folded IFP2 (null: the uniform
// weight c / (1 - c)): g[i] bounds the L1 mass that a unit of residual left at i would
// still add to the exact vector, q[i] the weight of a unit pushed from i into the
// non-dangling vertices (the mean of g over i's valid out-neighbours per deg(i)).
struct ErrWeights {
    const float *g;
    const float *q;
};

// A scatter item of a list sweep: a vertex with at most kLaneEdges valid out-edges is
// one lane's work; a longer row is cut into chunks of kChunkEdges edges, one wave's each.
constexpr int kLaneEdges = 16;
constexpr int kChunkEdges = 1024;
// Device buffers of list sweeps (capacities: nN frontier entries per list, nN lane
// items, nN + valid edges / kChunkEdges wave items).
template <typename T>
struct ListBufs {
    int32_t *f[2];         // frontier lists by sweep parity (vertex ids, unordered)
    int32_t *lane_v;       // lane items: vertex
    T *lane_w;             //   push weight c v / deg
    int32_t *wave_v;       // wave items: vertex
    int32_t *wave_c;       //   chunk index within the row
    T *wave_w;             //   push weight
};

// Control block of a batch of B <= kMaxBatch vectors (see Ctl).
constexpr int kMaxBatch = 16;
struct alignas(128) CtlB {
    int32_t stop_after;             // sweeps with index > stop_after do nothing
    int32_t use_pull;
    int32_t pull_sweeps;
    int32_t pad0;
    int32_t col_stop[kMaxBatch];    // column j reserves only in sweeps <= col_stop[j]
    int32_t col_sweeps[kMaxBatch];
    double sx[kMaxBatch];
    double last_bound[kMaxBatch];
    unsigned long long tot_pushes[kMaxBatch], tot_edges[kMaxBatch];
    unsigned long long tot_traversed;
    double fin_sum[kMaxBatch], fin_sn[kMaxBatch];
};

// sources of a batch (original ids; kSrcUnused = unused column, kSrcUniform =
// global PageRank column), passed by value
constexpr int32_t kSrcUnused = -1, kSrcUniform = -2;
struct SrcSet {
    int32_t s[kMaxBatch];
};
// output vector of each column (device pointers), passed by value
struct OutSet {
    double *p[kMaxBatch];
};

// Per-graph state of a multi-graph solve (device memory, one entry per graph).
// fin_sum and fin_sn are adjacent, and so are the five acc entries: the
// kernels accumulate into them as runs of doubles.
struct alignas(8) SetG {
    double c;             // damping factor of this graph
    double xi;            // push threshold (units where h0 = 1 per vertex)
    double sx;            // total mass sum(pibar + h) + untouched dangling mass
    double last_bound;    // bound certified at the last reserve
    double fin_sum, fin_sn;
    double acc[5];        // this sweep: inactive residual, mass to N, sx growth, pushes, pushed edges
    double sn;            // ordered sweeps: residual left on the non-dangling vertices, summed directly
    double m_nn;          // edges between non-dangling vertices (what a gather of this graph reads)
    unsigned long long tot_pushes, tot_edges;
    int32_t stop_after;   // last sweep whose scatter counts (INT_MAX while running)
    int32_t sweeps;
};

// Graph-set sweeps: per merge-path tile the first and last graph of its rows,
// so that tiles of graphs that stopped are skipped (all null for one graph).
struct TileSkip {
    const uint2 *tgr = nullptr;  // [tiles]
    const SetG *gs = nullptr;
};

// Optional timing of one sweep-kernel launch: the start / stop events are taken
// by the launch itself (no separate event records around it).
struct KernelEvents {
    hipEvent_t a = nullptr, b = nullptr;
};

struct Trace {
    unsigned long long cnt[kMaxTrace];
    unsigned long long edges[kMaxTrace];
    double sn[kMaxTrace];
    double bound[kMaxTrace];
};

// In-edge lists for the sweeps t >= t_start: only sources whose unreferenced
// depth is >= t_start (the others can no longer push).  Epoch 0 is the full list.
struct Epoch {
    int32_t t_start = 0;
    uint32_t *in_ptr = nullptr;  // [n + 1] (N targets first)
    int32_t *in_src = nullptr;
    int64_t edges_all = 0, edges_nn = 0;
    MPPlan pull_all, pull_nn;
};

// Device-resident graph: vertices relabelled so that the n_N non-dangling
// vertices come first ([0, n_N), original order kept), dangling after.
struct Graph {
    int64_t n = 0, m = 0;
    int32_t nN = 0, nD = 0;       // swept prefix [0, nN); deferred vertices [nN, n), nD = n - nN
    // PR_PEEL: weakly dangling vertices [nN, nN + nP) of the deferred region, by level from
    // the highest down; the rows of deg, rp_nn and rp_nd cover them too (nN + nP rows)
    int32_t nP = 0;
    std::vector<int32_t> lvl_lo;   // first new id of each deferred block (levels, then dangling), then n
    std::vector<MPPlan> lvl_pull;  // gather plan of each block's in-edges
    int64_t mNN = 0, mND = 0, n_unref = 0;
    int32_t *perm = nullptr;      // new id -> original id, [n]
    int32_t *newid = nullptr;     // original id -> new id, [n]
    int32_t *deg = nullptr;       // out-degree of non-dangling vertices, [nN + nP]
    uint32_t *rp_nn = nullptr;    // CSR of edges N -> N, [nN + nP + 1]
    int32_t *col_nn = nullptr;    // [mNN]
    uint32_t *rp_nd = nullptr;    // CSR of edges into the deferred region, [nN + nP + 1]
    int32_t *col_nd = nullptr;    // [mND]
    uint32_t *in_ptr = nullptr;   // in-edges of every target (N targets first), [n + 1]
    int32_t *in_src = nullptr;    // [m]
    MPPlan push_nn, push_nd, pull_all, pull_nn, pull_nd;
    // merge-path plans with tiles of (kBlock / B) * kMPK items for the batched kernels
    // of width B = 8 (index 0) and 16 (index 1), built on the first batched solve
    std::mutex bp_mu;
    bool bp_ready[2] = {false, false};
    std::vector<MPPlan> bp_pull_nn[2];  // per epoch
    MPPlan bp_pull_nd[2], bp_push_nn[2];
    // ordered sweeps of the batched kernels: per width, the gather plans of the vertex
    // groups' in-edges over the rows each group reaches ([epoch][group], sharing the
    // lists of grp_pull_rows), and per vertex the share of its push that stays residual
    // to the end of an ordered sweep (launch_amp_qle with unit weights); built for the
    // vertex groups of version bp_grp_version and owned with the groups (grp_allocs)
    std::vector<std::vector<MPPlan>> bp_grp[2];
    int64_t bp_grp_version[2] = {-1, -1};
    float *bp_qle = nullptr;
    int64_t bp_qle_version = -1;
    int32_t *depth = nullptr;     // unreferenced depth of non-dangling vertices, [nN + nP] (peeled: infinite)
    int32_t max_depth = -1;       // largest finite depth
    std::vector<Epoch> epochs;    // epochs[0] aliases the full in-edge lists
    int32_t tile_k = kMPK;        // merge-path items per thread of the sweep tiles
    // ordered sweeps: non-dangling sources split into groups of equal N -> N out-edges
    // (group g = [grp[g], grp[g + 1])), and per epoch the gather plans of each group's
    // in-edges: over the non-dangling rows (IFP2) and over all rows (IFP1), one list
    // serving both since the non-dangling rows come first
    std::vector<int32_t> grp;
    bool prefer_ordered = true;                     // set by the autotuner
    // batched solves (PPR batches, the server's batched runs) turn to ordered sweeps once
    // dense: -1 not measured (they do), 0 / 1 as the autotuner measured (see tune_impl)
    int32_t batch_order = -1;
    std::vector<std::vector<MPPlan>> grp_pull;      // [epoch][group], rows [0, nN)
    std::vector<std::vector<MPPlan>> grp_pull_all;  // [epoch][group], rows [0, n)
    // the same gathers over only the rows each group reaches (MPPlan::rid)
    std::vector<std::vector<MPPlan>> grp_pull_rows, grp_pull_all_rows;
    bool group_rows = true;                         // ordered sweeps use those (set by the autotuner)
    int64_t device_bytes = 0;
    double seconds_upload = 0, seconds_split = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<void *> allocs;
    std::vector<void *> grp_allocs;  // the vertex groups' lists and plans (rebuilt by the autotuner)
    int64_t grp_bytes = 0;
    // cached solve workspace
    std::mutex ws_mu;
    bool ws_busy = false;
    int32_t users = 0;    // solves and servers using the graph (guarded by ws_mu)
    bool tuning = false;  // the autotuner is rebuilding the plans (guarded by ws_mu)
    void *ws_mem = nullptr;
    size_t ws_bytes = 0;
    void *ws_hctl = nullptr;  // pinned host control block that goes with ws_mem
    // error weights of IFP2's stop rule, per damping factor (built by the first solve with
    // that factor, device arrays over [0, nN) owned by the graph)
    struct Amp {
        double c;
        float *g, *q;
        double seconds;  // time taken to build them (charged as preprocessing)
        // q restricted to the out-neighbours in the vertex's own group or an earlier one,
        // for the vertex groups of version qle_version (see launch_amp_qle)
        float *qle = nullptr;
        int64_t qle_version = -1;
        double qle_seconds = 0.0;  // time taken to build qle (charged as preprocessing)
    };
    int64_t grp_version = 0;  // bumped whenever the vertex groups are rebuilt
    std::mutex amp_mu;
    std::vector<Amp> amp;
    std::vector<uint64_t> dangling_bits;  // host bitmap over original ids: no out-edges
    bool dangling(int64_t v) const { return (dangling_bits[(size_t)v >> 6] >> (v & 63)) & 1u; }
};

// Ordered sweeps of a batched solve of width B (slot 0: 8, 1: 16) are possible: the graph
// has vertex groups, prefers ordered sweeps (for batches too, unless the autotuner found
// them slower there), and its batched group plans are current.
inline bool batch_ordered_ready(const Graph &G, int slot) {
    const int ng = (int)G.grp.size() - 1;
    return ng > 1 && ng <= kMaxGroups && G.prefer_ordered && G.batch_order != 0 && G.bp_qle != nullptr &&
           G.bp_qle_version == G.grp_version && G.bp_grp_version[slot] == G.grp_version &&
           G.bp_grp[slot].size() == G.epochs.size();
}
// workgroups of each group's reserve in a batched ordered sweep of width B (about four
// (vertex, column) entries per thread, at most kGroupBlocks)
inline GroupBlocks batch_group_blocks(const Graph &G, int B) {
    GroupBlocks gb{};
    gb.stride = kGroupBlocks;
    for (size_t q = 0; q + 1 < G.grp.size() && q < (size_t)kMaxGroups; ++q) {
        const int64_t work = ((int64_t)G.grp[q + 1] - G.grp[q]) * B;
        const int64_t b = (work + 4 * kBlock - 1) / (4 * kBlock);
        gb.nb[q] = (int32_t)(b < 1 ? 1 : (b > kGroupBlocks ? kGroupBlocks : b));
    }
    return gb;
}

// host helpers for the query server (pr_host.hip: errors; pr_solve.hip: batched plans)
pr_status set_error(pr_status st, const std::string &msg);
void clear_error();
pr_status batch_plans(Graph &G, int B, hipStream_t s);  // B = 8 or 16

// ---- kernel launchers (pr_kernels.hip) ----
hipError_t launch_check_cols(const int32_t *col, int64_t m, int64_t n, unsigned int *bad, hipStream_t s);
hipError_t launch_degree_class(const int64_t *rp64, int64_t n, uint32_t *isN, hipStream_t s);
hipError_t launch_indegree(const int32_t *col, int64_t m, uint32_t *indeg, hipStream_t s);
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
// the rows r < R of a gather plan that have an edge (cnt[r] > 0): flag[r] = 1 or 0; after an
// exclusive scan pos of flag, rid[pos[r]] = r and rp[pos[r]] = off[r] for those rows, and
// rp[pos[R]] = off[R] (off: the plan's R + 1 edge offsets)
hipError_t launch_row_flags(int32_t R, const uint32_t *cnt, uint32_t *flag, hipStream_t s);
hipError_t launch_row_fill(int32_t R, const uint32_t *cnt, const uint32_t *pos, const uint32_t *off, int32_t *rid,
                           uint32_t *rp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);
hipError_t launch_relabel(const uint32_t *isN, const uint32_t *rankN, int64_t n, int32_t nN, int32_t *newid,
                          int32_t *perm, hipStream_t s);
hipError_t launch_count_nn(const int64_t *rp64, const int32_t *col, const uint32_t *isN, const int32_t *perm,
                           int32_t nN, uint32_t *cnt_nn, uint32_t *cnt_nd, int32_t *deg, hipStream_t s);
hipError_t launch_split_rows(const int64_t *rp64, const int32_t *col, const uint32_t *isN, const int32_t *newid,
                             const int32_t *perm, int32_t nN, const uint32_t *rp_nn, int32_t *col_nn,
                             const uint32_t *rp_nd, int32_t *col_nd, hipStream_t s);
hipError_t launch_permute_u32(const uint32_t *in_old, const int32_t *perm, int64_t n, uint32_t *out_new,
                              hipStream_t s);
hipError_t launch_fill_csc(const uint32_t *rp, const int32_t *col, int32_t R, uint32_t *cursor, int32_t *in_src,
                           hipStream_t s);
// PR_PEEL phase 2: w2[v] = c xD[v - nN] / deg[v] for the peeled block [lo, hi)
hipError_t launch_peel_w2(int32_t lo, int32_t hi, int32_t nN, const double *xD, const int32_t *deg, double c,
                          double *w2, hipStream_t s);
hipError_t launch_count_zero(const uint32_t *a, int64_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_plan(MPPlan &p, hipStream_t s);
hipError_t launch_depth_init(int32_t nN, const uint32_t *in_ptr, uint32_t *rem, int32_t *depth, int32_t *q,
                             uint32_t *qcount, hipStream_t s);
hipError_t launch_depth_step(const int32_t *q, uint32_t qsize, const uint32_t *rp_nn, const int32_t *col_nn,
                             uint32_t *rem, int32_t *depth, int32_t round, int32_t *next, uint32_t *ncount,
                             hipStream_t s);
// every in-edge list sorted by source id (pr_sort.hip); synchronises the stream
hipError_t sort_in_lists(int64_t n, int64_t m, const uint32_t *in_ptr, int32_t *in_src, hipStream_t s);
// in-edges whose source has depth >= t0, lies in [slo, shi) and, when grp is given,
// belongs to vertex group q (grp[u] == q)
hipError_t launch_live_count(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                             int32_t t0, int32_t slo, int32_t shi, uint32_t *cnt, hipStream_t s,
                             const uint8_t *grp = nullptr, int32_t q = 0);
hipError_t launch_live_fill(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                            int32_t t0, int32_t slo, int32_t shi, const uint32_t *out_ptr, int32_t *out_src,
                            hipStream_t s, const uint8_t *grp = nullptr, int32_t q = 0);

// solve kernels
struct InitArgs {
    int64_t n;
    int32_t nN;
    int uniform;            // p == NULL
    const double *p;        // original order (device) when !uniform
    double pscale;          // 1 / sum(p)
    const int32_t *perm;
    int32_t source;         // >= 0: single-source PPR (original id): p = e_source
};
template <typename T>
hipError_t launch_init_ifp(const InitArgs &a, T *h, double *pibar, hipStream_t s);
template <typename T>
hipError_t launch_reserve(int t, Ctl *ctl, Trace *tr, int32_t nN, T *h, T *w, double *pibar, const int32_t *deg,
                          const uint32_t *rp_nn, double c, double xi, int ifp2, ErrWeights ew, double kb,
                          int stop_l1, double tol, unsigned long long pull_edges_thr, int force,
                          unsigned long long pull_edges, double *part, hipStream_t s);
// ordered sweeps: reserve of the non-dangling range [lo, hi) into nbg workgroup
// partials (5 * nbg doubles at part), the residual left behind weighted by ew.g and the
// pushed mass by ew.q; after all groups, k_decide_gs (bookkeep: S_N from those sums, with
// ew.q the reach-restricted weights of launch_amp_qle; else from a k_sum_h pass)
template <typename T>
hipError_t launch_reserve_range(int t, Ctl *ctl, int32_t lo, int32_t hi, T *h, T *w, double *pibar,
                                const int32_t *deg, const uint32_t *rp_nn, double c, double xi, int ifp2, int nbg,
                                ErrWeights ew, double *part, hipStream_t s);
template <typename T>
hipError_t launch_decide_gs(int t, Ctl *ctl, Trace *tr, int32_t nN, const T *h, int ng, const GroupBlocks &gb,
                            const double *part, double *part_s, double c, const float *g, double kb, int stop_l1,
                            double tol, unsigned long long pull_thr, unsigned long long pull_edges, int bookkeep,
                            hipStream_t s);
template <typename T>
hipError_t launch_push(int t, const Ctl *ctl, const MPPlan &p, const T *w, T *h, int check_mode, hipStream_t s,
                       TileSkip skip = TileSkip(), KernelEvents ev = KernelEvents());
template <typename WT, typename OT>
hipError_t launch_pull(int t, const Ctl *ctl, const MPPlan &p, const WT *w, OT *out, int check_mode,
                       hipStream_t s, TileSkip skip = TileSkip(), KernelEvents ev = KernelEvents());
template <typename T>
hipError_t launch_phase2_prep(const InitArgs &a, const T *h, const double *pibar, const int32_t *deg, double c,
                              int literal, double *w2, double *xD, hipStream_t s);
template <typename T>
hipError_t launch_final_ifp(Ctl *ctl, const InitArgs &a, const T *h, const double *pibar, const double *xD,
                            int ifp2, int literal, const float *g, double *out, double *part, hipStream_t s);
// power method
template <typename WT>
hipError_t launch_power_prescale(int t, Ctl *ctl, const InitArgs &a, double *x, double *acc, WT *y,
                                 const int32_t *deg, double c, double tol, double *part, hipStream_t s);
hipError_t launch_power_init(const InitArgs &a, double *x, double *acc, hipStream_t s);
hipError_t launch_final_x(Ctl *ctl, const InitArgs &a, const double *x, double *out, double *part, hipStream_t s);
// a-posteriori check of the normalised output `out` (original order, device): fills
// vctl->ver_r / ver_err / ver_sum, and ver_rf when the stop-rule weights g of factor c
// (ErrWeights::g, over the first nN vertices; rp_nn their non-dangling out-degrees) are
// given; x, acc: n doubles, y: doubles for every vertex with out-edges; *depth receives
// the reduction depth used for the rounding bound
hipError_t launch_verify(Ctl *vctl, const InitArgs &a, const double *out, double *x, double *acc, double *y,
                         const int32_t *deg, const MPPlan &pull_all, const uint32_t *in_ptr, double c, const float *g,
                         int32_t nN, const uint32_t *rp_nn, double *part, double *depth, hipStream_t s);
// zero-fill kernels (used instead of memset nodes on the solve stream)
hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t count, hipStream_t s);
// error weights of IFP2's stop rule (ErrWeights) for damping c: iterations of the
// future-mass recursion from its upper bound 1 / (1 - c) over the N -> N out-edges
// (plan push_nn), each an upper bound; f and acc: nN doubles of scratch
// qle[u] = (sum of g over u's non-dangling out-neighbours in u's vertex group or an earlier
// one) / deg(u), rounded up: the weight of mass u pushes in an ordered sweep that is still
// residual when the sweep ends (a later group takes the rest within the sweep); with g
// null, unit weights (the share of u's push that stays residual)
hipError_t launch_amp_qle(int32_t nN, const uint32_t *rp_nn, const int32_t *col_nn, const int32_t *deg,
                          const float *g, const GroupEnds &ge, float *qle, hipStream_t s);
hipError_t launch_amp_weights(int32_t nN, const MPPlan &push_nn, const int32_t *deg, const uint32_t *rp_nn,
                              double c, int iters, double *f, double *acc, float *g, float *q, hipStream_t s);
// kernel launches of the calling thread so far (counted by the launchers)
extern thread_local int64_t t_kernel_launches;
// list sweeps (compacted frontier; IFP1 / IFP2 with non-negative residuals)
// frontier list of sweep t (slot t & 1) from every non-dangling h_i > xi, and the
// residual on the non-dangling vertices into ctl->sn_last; the list counters must be zero
template <typename T>
hipError_t launch_compact(Ctl *ctl, int slot, int32_t nN, const T *h, double xi, int32_t *f, const int32_t *deg,
                          const uint32_t *rp_nn, int ifp2, const float *g, double *part, hipStream_t s);
// reserve + decision of list sweep t over the frontier list of slot t & 1
template <typename T>
hipError_t launch_reserve_list(int t, Ctl *ctl, Trace *tr, const ListBufs<T> &lb, T *h, double *pibar,
                               const int32_t *deg, const uint32_t *rp_nn, double c, double xi, int ifp2,
                               ErrWeights ew, double kb, int stop_l1, double tol, double *part, hipStream_t s);
// scatter of list sweep t; targets whose residual rises above xi form the frontier of t + 1
template <typename T>
hipError_t launch_push_list(int t, Ctl *ctl, const ListBufs<T> &lb, T *h, const int32_t *deg, const uint32_t *rp_nn,
                            const int32_t *col_nn, const uint32_t *rp_nd, const int32_t *col_nd, double xi, int ifp2,
                            hipStream_t s);
hipError_t launch_validate_p(const double *p, int64_t n, double *sum_bad, hipStream_t s);
hipError_t launch_unit_vector(double *out, int64_t n, int64_t src, hipStream_t s);

// multi-graph solve (pr_set.hip); offN / offD: k + 1 segment offsets of the
// graphs in the non-dangling and dangling regions of the union
template <typename T>
hipError_t launch_set_init(int64_t n, int32_t nN, T *h, double *pibar, hipStream_t s);
// reserve over `len` positions: position p of graph g (pos_off[g] <= p < pos_off[g + 1])
// is vertex p + base[g] (base NULL: 0, positions are the non-dangling vertices)
template <typename T>
hipError_t launch_set_reserve(int t, const Ctl *ctl, SetG *gs, const int32_t *pos_off, const int32_t *base,
                              int32_t k, int32_t len, T *h, T *w, double *pibar, const int32_t *deg,
                              const uint32_t *rp_nn, hipStream_t s);
// ordered sweeps: per running graph, sum |h| over its non-dangling vertices into SetG::sn
template <typename T>
hipError_t launch_set_sum_h(int t, const Ctl *ctl, SetG *gs, const int32_t *offN, int32_t k, int32_t nN,
                            const T *h, hipStream_t s);
hipError_t launch_set_tile_graphs(const MPPlan &p, const int32_t *offN, int32_t k, uint2 *out, hipStream_t s);
hipError_t launch_set_decide(int t, Ctl *ctl, SetG *gs, int32_t k, int stop_l1, double tol, double live_frac,
                             int force, int ordered, hipStream_t s);
template <typename T>
hipError_t launch_set_phase2_prep(int64_t n, int32_t nN, const SetG *gs, const int32_t *offN, int32_t k,
                                  const T *h, const double *pibar, const int32_t *deg, double *w2, double *xD,
                                  hipStream_t s);
template <typename T>
hipError_t launch_set_final(int64_t n, int32_t nN, SetG *gs, const int32_t *offN, const int32_t *offD, int32_t k,
                            const int32_t *perm, const T *h, const double *pibar, const double *xD, double *out,
                            hipStream_t s);

// warm start (pr_warm.hip): state arrays in original ids
template <typename T>
hipError_t launch_warm_import(Ctl *ctl, int64_t n, int32_t nN, const int32_t *perm, const double *st_pibar,
                              const double *st_h, T *h, double *pibar, double *pibar0, double *xD0, double *hD0,
                              double *part, hipStream_t s);
template <typename T>
hipError_t launch_warm_phase2_prep(int32_t nN, int32_t nD, const T *h, const double *pibar, const double *pibar0,
                                   const int32_t *deg, double c, const double *xD0, const double *hD0, double *w2,
                                   double *w3, double *xD, double *hDn, hipStream_t s);
template <typename T>
hipError_t launch_warm_export(int64_t n, int32_t nN, const int32_t *perm, const T *h, const double *pibar,
                              const double *hDn, double *st_pibar, double *st_h, hipStream_t s);
struct Graph;
hipError_t launch_state_update(const int32_t *src, int64_t count, const Graph &g_old, const Graph &g_new, double c,
                               const double *st_pibar, double *st_h, hipStream_t s);

// batched IFP2 (pr_batch.hip)
template <typename T, int B>
hipError_t launch_init_b(int64_t n, int32_t nN, const int32_t *perm, const SrcSet &src, uint32_t mask, T *h,
                         double *pibar, hipStream_t s);
template <typename T, int B>
hipError_t launch_reserve_b(int t, CtlB *ctl, int32_t nN, T *h, T *w, double *pibar, const int32_t *deg,
                            const uint32_t *rp_nn, double c, double xi, int stop_l1, double tol, double pull_thr,
                            int force, unsigned long long pull_edges, double *part, hipStream_t s);
// the reserve of rows [lo, hi) in an ordered sweep (nb workgroups, 5 partial rows of B
// columns from part; qle: the share of each vertex's push that stays residual to the end
// of the sweep), and the decision after all groups have reserved and gathered
template <typename T, int B>
hipError_t launch_reserve_range_b(int t, CtlB *ctl, int32_t lo, int32_t hi, T *h, T *w, double *pibar,
                                  const int32_t *deg, const uint32_t *rp_nn, double c, double xi, const float *qle,
                                  int nb, double *part, hipStream_t s);
template <int B>
hipError_t launch_decide_gs_b(int t, CtlB *ctl, int ngr, const GroupBlocks &gb, const double *part, double *sums,
                              double c, int stop_l1, double tol, double pull_thr, unsigned long long sweep_edges,
                              hipStream_t s);
template <typename T, int B>
hipError_t launch_push_b(int t, const CtlB *ctl, const MPPlan &p, const T *w, T *h, int check_mode, hipStream_t s);
template <typename WT, typename OT, int B>
hipError_t launch_pull_b(int t, const CtlB *ctl, const MPPlan &p, const WT *w, OT *out, int check_mode,
                         hipStream_t s);
template <typename T, int B>
hipError_t launch_phase2_b(int64_t n, int32_t nN, const int32_t *perm, const SrcSet &src, const T *h,
                           const double *pibar, const int32_t *deg, double c, double *w2, double *xD,
                           const MPPlan &pull_nd, hipStream_t s);
template <typename T, int B>
hipError_t launch_final_b(CtlB *ctl, int64_t n, int32_t nN, const int32_t *perm, uint32_t mask, const OutSet &out,
                          const T *h, const double *pibar, const double *xD, double *part, hipStream_t s);

}  // namespace prk

struct pr_graph {
    prk::Graph g;
};
