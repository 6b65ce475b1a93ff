// pr_batch.hip -- IFP2 for B personalization vectors at once (single-source PPR
// batches).  Vectors are stored column-interleaved, element (v, j) at v * B + j,
// so one random in-edge gather fetches the B weights of a source as one
// contiguous 4B / 8B * B segment: the cost of the random access is shared by B
// queries.  Each column keeps its own stop decision; a stopped column is frozen.
#include "pr_device.h"

namespace prk {
namespace {

// per-column sum over the threads of a workgroup that hold column tid % B;
// results valid in threads 0 .. B-1 (column = threadIdx.x)
template <int B>
__device__ __forceinline__ double block_sum_cols(double v, double *sbuf /* [kBlock / W * B] */) {
#pragma unroll
    for (int o = B; o < W; o <<= 1) v += __shfl_xor(v, o, W);
    __syncthreads();
    if (lane_id() < B) sbuf[(threadIdx.x / W) * B + lane_id()] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < B) {
#pragma unroll
        for (int k = 0; k < kBlock / W; ++k) r += sbuf[k * B + threadIdx.x];
    }
    return r;
}

// initial residual of column j at vertex v: n at the source (p = e_s), 1 everywhere
// for a global PageRank column (p = e / n), 0 for an unused column
template <typename T>
__device__ __forceinline__ double h0_col(int32_t s, int32_t orig, int64_t n) {
    if (s == kSrcUniform) return 1.0;
    return (s >= 0 && orig == s) ? (double)n : 0.0;
}

// (re)initialise the columns in `mask`; the others are left untouched
template <typename T, int B>
__global__ void k_init_b(int64_t n, int32_t nN, const int32_t *perm, SrcSet src, uint32_t mask, T *h,
                         double *pibar) {
    const int64_t total = n * B;
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kBlock) {
        const int j = (int)(idx % B);
        if (!((mask >> j) & 1u)) continue;
        const int64_t v = idx / B;
        h[idx] = (T)h0_col<T>(src.s[j], perm[v], n);
        if (v < nN) pibar[idx] = 0.0;
    }
}

// Reserve step of rows [lo, hi) for every live column (see k_reserve): partials per
// column, layout part[(q * B + j) * nb + block] for q = inactive residual, mass sent to
// non-dangling vertices, active vertices, their edges, and with qle (an ordered sweep's
// group) the pushed mass weighted by qle: the share of a vertex's push that lands in its
// own group or an earlier one, where it stays residual to the end of the sweep.
template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_reserve_b(int t, const CtlB *ctl, int32_t lo, int32_t hi, T *h, T *w,
                                                      double *pibar, const int32_t *deg, const uint32_t *rp_nn,
                                                      double c, T xi, const float *qle, double *part) {
    if (t > ctl->stop_after) return;
    const int j = threadIdx.x % B;  // the grid stride is a multiple of B: a thread keeps its column
    const bool live = t <= ctl->col_stop[j];
    double inact = 0.0, pred = 0.0, cnt = 0.0, edges = 0.0, stay = 0.0;
    const int64_t first = (int64_t)lo * B, total = (int64_t)hi * B;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // one (vertex, column) entry whose inputs are loaded (dg, r0, r1, pb, ql read only when active)
    auto take = [&](int64_t idx, T hv, int32_t dg, uint32_t r0, uint32_t r1, double pb, float ql) {
        if (live && hv > xi) {
            const uint32_t dnn = r1 - r0;
            const double val = (double)hv;
            pibar[idx] = pb + val;
            h[idx] = (T)0;
            w[idx] = (T)(c * val / (double)dg);
            pred += val * ((double)dnn / (double)dg);
            stay += val * (double)ql;
            cnt += 1.0;
            edges += (double)dnn;
        } else {
            w[idx] = (T)0;
            inact += (double)hv;
        }
    };
    int64_t idx = first + blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (ctl->use_pull || total - first <= stride) {
        // dense frontier, or about one entry per thread (uniform over the grid): an
        // entry's degree, row offsets and pibar are loaded with its residual, two
        // entries per iteration, instead of after the test; sums run in the same order
        for (; idx < total; idx += 2 * stride) {
            const int64_t i2 = idx + stride;
            const bool two = i2 < total;
            const int64_t v = idx / B;
            const T hv = h[idx];
            const int32_t dg = deg[v];
            const uint32_t r0 = rp_nn[v], r1 = rp_nn[v + 1];
            const double pb = pibar[idx];
            const float ql = qle ? qle[v] : 0.0f;
            T hv2 = (T)0;
            int32_t dg2 = 1;
            uint32_t s0 = 0, s1 = 0;
            double pb2 = 0.0;
            float ql2 = 0.0f;
            if (two) {
                const int64_t v2 = i2 / B;
                hv2 = h[i2];
                dg2 = deg[v2];
                s0 = rp_nn[v2];
                s1 = rp_nn[v2 + 1];
                pb2 = pibar[i2];
                ql2 = qle ? qle[v2] : 0.0f;
            }
            take(idx, hv, dg, r0, r1, pb, ql);
            if (two) take(i2, hv2, dg2, s0, s1, pb2, ql2);
        }
    } else {
        for (; idx < total; idx += stride) {
            const int64_t v = idx / B;
            const T hv = h[idx];
            if (live && hv > xi) take(idx, hv, deg[v], rp_nn[v], rp_nn[v + 1], pibar[idx], qle ? qle[v] : 0.0f);
            else take(idx, hv, 0, 0, 0, 0.0, 0.0f);
        }
    }
    __shared__ double sd[kBlock / W * B];
    const double r0 = block_sum_cols<B>(inact, sd);
    const double r1 = block_sum_cols<B>(pred, sd);
    const double r3 = block_sum_cols<B>(cnt, sd);
    const double r4 = block_sum_cols<B>(edges, sd);
    const double r5 = qle ? block_sum_cols<B>(stay, sd) : 0.0;  // qle is uniform over the grid
    if (threadIdx.x < B) {
        const int nb = gridDim.x, b = blockIdx.x, jj = threadIdx.x;
        part[(0 * B + jj) * nb + b] = r0;
        part[(1 * B + jj) * nb + b] = r1;
        part[(2 * B + jj) * nb + b] = r3;
        part[(3 * B + jj) * nb + b] = r4;
        if (qle) part[(4 * B + jj) * nb + b] = r5;
    }
}

// Management step for B columns (one workgroup).  Column j stops after the
// sweep whose scatter certifies its L1 bound (or before a sweep that moves
// nothing); the batch stops when every column has.
template <int B>
__global__ __launch_bounds__(1024) void k_decide_b(int t, CtlB *ctl, int nb, const double *part, double c,
                                                     int stop_l1, double tol, double pull_thr, int force,
                                                     unsigned long long pull_edges) {
    if (t > ctl->stop_after) return;
    __shared__ double s_sum[4 * B];
    // one wave per partial row (4B rows of nb <= kRedBlocks entries); a lane loads
    // all its entries of a row before adding them, in index order
    constexpr int kRounds = kRedBlocks / W;
    const int wv = threadIdx.x / W;
    for (int r = wv; r < 4 * B; r += blockDim.x / W) {
        const double *row = part + (int64_t)r * nb;
        double x[kRounds];
#pragma unroll
        for (int q = 0; q < kRounds; ++q) {
            const int b = lane_id() + q * W;
            x[q] = b < nb ? row[b] : 0.0;
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kRounds; ++q) s += x[q];
        s = wave_sum(s);
        if (lane_id() == 0) s_sum[r] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double k = 2.0 * c / (1.0 - c);
    bool any_moved = false, any_next = false;
    double total_edges = 0.0;
    for (int j = 0; j < B; ++j) {
        if (t > ctl->col_stop[j]) continue;  // frozen column
        const double a_in = s_sum[0 * B + j], a_pr = s_sum[1 * B + j];
        const double a_c = s_sum[2 * B + j], a_e = s_sum[3 * B + j];
        if (a_c == 0.0) {
            ctl->col_stop[j] = t - 1;
            ctl->last_bound[j] = k * a_in / ctl->sx[j];
            continue;
        }
        any_moved = true;
        total_edges += a_e;
        const double sn = a_in + c * a_pr;
        const double sx = ctl->sx[j] + c * a_pr;  // IFP2: the mass that stays on non-dangling vertices
        ctl->sx[j] = sx;
        const double bound = k * sn / sx;
        ctl->last_bound[j] = bound;
        ctl->col_sweeps[j] = t + 1;
        ctl->tot_pushes[j] += (unsigned long long)a_c;
        ctl->tot_edges[j] += (unsigned long long)a_e;
        if (stop_l1 && bound <= tol) ctl->col_stop[j] = t;
        else any_next = true;
    }
    const int pull = force == 1 ? 0 : (force == 2 ? 1 : (total_edges >= pull_thr ? 1 : 0));
    ctl->use_pull = pull;
    if (any_moved) {
        ctl->pull_sweeps += pull;
        ctl->tot_traversed += pull ? pull_edges : (unsigned long long)total_edges;
    }
    if (!any_next) ctl->stop_after = any_moved ? t : t - 1;
}

// Row sums of an ordered sweep's reserve partials: workgroup r sums row r % (5B) of
// group r / (5B) (gb.nb[q] entries, every load issued before the first add, added in
// index order) into sums[r].
template <int B>
__global__ __launch_bounds__(kBlock) void k_rowsum_gs_b(int t, const CtlB *ctl, GroupBlocks gb, const double *part,
                                                        double *sums) {
    if (t > ctl->stop_after) return;
    constexpr int kRounds = kGroupBlocks / kBlock;
    const int q = blockIdx.x / (5 * B), r = blockIdx.x % (5 * B);
    const int nb = gb.nb[q];
    const double *row = part + (size_t)5 * B * gb.stride * q + (size_t)r * nb;
    double x[kRounds];
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        const int b = threadIdx.x + k * kBlock;
        x[k] = b < nb ? row[b] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) v += x[k];
    __shared__ double sd[kBlock / W];
    v = block_sum(v, sd);
    if (threadIdx.x == 0) sums[blockIdx.x] = v;
}

// Management step of an ordered sweep for B columns (one workgroup), after every group
// has reserved and gathered.  Column j's residual left on the non-dangling vertices is
// what the reserves left behind plus c times the pushed mass that landed in the pushing
// vertex's own group or an earlier one (mass pushed into a later group met that group's
// reserve in the same sweep: taken, or counted as left behind); the stop rules are
// those of k_decide_b.
template <int B>
__global__ __launch_bounds__(kBlock) void k_decide_gs_b(int t, CtlB *ctl, int ngr, const double *sums, double c,
                                                        int stop_l1, double tol, double pull_thr,
                                                        unsigned long long sweep_edges) {
    if (t > ctl->stop_after) return;
    __shared__ double s5[5 * B];
    if (threadIdx.x < 5 * B) {
        double v = 0.0;
        for (int q = 0; q < ngr; ++q) v += sums[(size_t)5 * B * q + threadIdx.x];
        s5[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double k = 2.0 * c / (1.0 - c);
    bool any_moved = false, any_next = false;
    double total_edges = 0.0;
    for (int j = 0; j < B; ++j) {
        if (t > ctl->col_stop[j]) continue;  // frozen column
        const double a_in = s5[0 * B + j], a_pr = s5[1 * B + j];
        const double a_c = s5[2 * B + j], a_e = s5[3 * B + j], a_st = s5[4 * B + j];
        if (a_c == 0.0) {
            ctl->col_stop[j] = t - 1;
            ctl->last_bound[j] = k * a_in / ctl->sx[j];
            continue;
        }
        any_moved = true;
        total_edges += a_e;
        const double sn = a_in + c * a_st;
        const double sx = ctl->sx[j] + c * a_pr;
        ctl->sx[j] = sx;
        const double bound = k * sn / sx;
        ctl->last_bound[j] = bound;
        ctl->col_sweeps[j] = t + 1;
        ctl->tot_pushes[j] += (unsigned long long)a_c;
        ctl->tot_edges[j] += (unsigned long long)a_e;
        if (stop_l1 && bound <= tol) ctl->col_stop[j] = t;
        else any_next = true;
    }
    // would a synchronous sweep gather (is the frontier dense)
    ctl->use_pull = total_edges >= pull_thr ? 1 : 0;
    if (any_moved) {
        ctl->pull_sweeps += 1;
        ctl->tot_traversed += sweep_edges;
    }
    if (!any_next) ctl->stop_after = any_moved ? t : t - 1;
}

// Scatter for B columns: a group of B lanes walks the merge-path items, lane j
// adds column j of the source's weight to column j of each target.
template <typename T, int B, int K>
__global__ __launch_bounds__(kBlock) void k_push_b(int t, const CtlB *ctl, int check_mode, const uint32_t *rp,
                                                   int32_t R, const int32_t *col, const uint2 *plan, uint32_t items,
                                                   int32_t ntiles, const T *w, T *h) {
    constexpr int G = kBlock / B;  // groups per workgroup
    constexpr int IPB = G * K;     // items per tile
    if (t > ctl->stop_after || (check_mode && ctl->use_pull)) return;
    __shared__ uint32_t s_end[IPB + 1];
    __shared__ int32_t s_col[IPB];
    __shared__ T s_w[(IPB + 1) * B];
    const uint32_t rp0 = rp[0];
    const int g = threadIdx.x / B, j = threadIdx.x % B;
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint2 a = plan[tile], b = plan[tile + 1];
        const int32_t i0 = (int32_t)a.x;
        const int32_t i1 = min((int32_t)b.x, R - 1);
        const uint32_t e0 = a.y, e1 = b.y;
        const int32_t nr = i1 - i0 + 1;
        int any = 0;
        for (int32_t kk = threadIdx.x; kk < nr; kk += kBlock) s_end[kk] = rp[i0 + 1 + kk] - rp0 + (uint32_t)(i0 + kk);
        for (int32_t q = threadIdx.x; q < nr * B; q += kBlock) {
            const T wv = w[(int64_t)i0 * B + q];
            s_w[q] = wv;
            any |= wv != (T)0;
        }
        any = __syncthreads_or(any);
        if (!any) continue;
        const int32_t ne = (int32_t)(e1 - e0);
        for (int32_t e = threadIdx.x; e < ne; e += kBlock) s_col[e] = col[e0 + e];
        __syncthreads();
        uint32_t d = min((uint32_t)(tile * IPB + g * K), items);
        const uint32_t dend = min(d + (uint32_t)K, items);
        if (d < dend) {
            int32_t lo = 0, hi = nr;
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (s_end[mid] < d) lo = mid + 1;
                else hi = mid;
            }
            int32_t k = lo;
            uint32_t et = rp0 + d - (uint32_t)(i0 + k);
            T wr = k < nr ? s_w[k * B + j] : (T)0;
            for (; d < dend; ++d) {
                if (d == s_end[k]) {
                    ++k;
                    wr = k < nr ? s_w[k * B + j] : (T)0;
                } else {
                    if (wr != (T)0) atomicAdd(h + (int64_t)s_col[et - e0] * B + j, wr);
                    ++et;
                }
            }
        }
        __syncthreads();
    }
}

// Gather for B columns: out[j of row r] += sum of w[j of source] over the row's
// in-edges.  The tile's B-wide weight segments are first gathered into LDS
// (consecutive lanes read consecutive columns of one source), then a group of
// B lanes walks the tile's items, lane j summing column j in FP64; rows shared
// by groups meet in an LDS accumulator (FP64, FP32 when the output is FP32: the
// sum is rounded to FP32 when it reaches the output anyway), and so do rows one
// group holds whole; the tile then writes all its rows out in one coalesced pass,
// rows shared by tiles through one global atomic per column and tile.  With rid, plan
// row r is target row rid[r] (a vertex group's gather over the rows it reaches).
template <typename WT, typename OT, int B, int K>
__global__ __launch_bounds__(kBlock) void k_pull_b(int t, const CtlB *ctl, int check_mode, const uint32_t *rp,
                                                   int32_t R, const int32_t *src, const uint2 *plan, uint32_t items,
                                                   int32_t ntiles, const int32_t *rid, const WT *w, OT *out) {
    constexpr int G = kBlock / B;
    constexpr int IPB = G * K;
    static_assert(IPB <= kBlock, "one row end per thread");
    using AccT = typename std::conditional<sizeof(OT) == 4, float, double>::type;
    if (t >= 0 && (t > ctl->stop_after || (check_mode && !ctl->use_pull))) return;
    __shared__ uint32_t s_end[IPB];
    __shared__ WT s_val[IPB * B];
    __shared__ AccT s_acc[IPB * B];
    const uint32_t rp0 = rp[0];
    const int g = threadIdx.x / B, j = threadIdx.x % B;
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint2 a = plan[tile], b = plan[tile + 1];
        const int32_t i0 = (int32_t)a.x;
        const int32_t i1 = min((int32_t)b.x, R - 1);
        const uint32_t e0 = a.y, e1 = b.y;
        // a tile of IPB items touches IPB + 1 rows only when all its items end rows (it
        // holds no edge): the last of them then has no item here and is left out
        const int32_t nr = min(i1 - i0 + 1, IPB);
        const uint32_t first = rp[i0];
        const int32_t ne = (int32_t)(e1 - e0);
        // Every load of the tile issues before the first LDS store: one row end per
        // thread (nr <= IPB <= kBlock), then K source ids (element q = e * B + column)
        // and K weights, indices clamped so that the loads are unconditional.
        const uint32_t rv = rp[i0 + 1 + min((int32_t)threadIdx.x, nr - 1)];
        int32_t sidx[K];
        WT v[K];
        if (ne > 0) {  // uniform over the workgroup
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int32_t q = threadIdx.x + r * kBlock;
                sidx[r] = src[e0 + min(q / B, ne - 1)];
            }
#pragma unroll
            for (int r = 0; r < K; ++r) v[r] = w[(int64_t)sidx[r] * B + j];
        }
        if ((int32_t)threadIdx.x < nr) s_end[threadIdx.x] = rv - rp0 + (uint32_t)(i0 + threadIdx.x);
        for (int32_t q = threadIdx.x; q < nr * B; q += kBlock) s_acc[q] = (AccT)0;
        if (ne > 0) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int32_t q = threadIdx.x + r * kBlock;
                if (q / B < ne) s_val[q] = v[r];
            }
        }
        __syncthreads();
        uint32_t d = min((uint32_t)(tile * IPB + g * K), items);
        const uint32_t dend = min(d + (uint32_t)K, items);
        if (d < dend) {
            int32_t lo = 0, hi = nr;
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (s_end[mid] < d) lo = mid + 1;
                else hi = mid;
            }
            int32_t k = lo;
            uint32_t et = rp0 + d - (uint32_t)(i0 + k);
            const uint32_t row_first = k == 0 ? first : s_end[k - 1] + rp0 + 1u - (uint32_t)(i0 + k);
            bool owned = et == row_first;
            bool touched = false;
            double acc = 0.0;
            for (; d < dend; ++d) {
                if (d == s_end[k]) {
                    if (touched) {
                        // a row this lane group holds whole has no other writer in the tile
                        if (owned) s_acc[k * B + j] = (AccT)acc;
                        else atomicAdd(s_acc + k * B + j, (AccT)acc);
                    }
                    acc = 0.0;
                    touched = false;
                    owned = true;
                    ++k;
                } else {
                    acc += (double)s_val[(et - e0) * B + j];
                    touched = true;
                    ++et;
                }
            }
            if (touched) atomicAdd(s_acc + k * B + j, (AccT)acc);
        }
        __syncthreads();
        for (int32_t q = threadIdx.x; q < nr * B; q += kBlock) {
            const double v = (double)s_acc[q];
            if (v == 0.0) continue;
            const int32_t k = q / B;
            // plan row i0 + k is target row rid[i0 + k] when the plan keeps only some rows
            OT *o = out + (rid ? (int64_t)rid[i0 + k] * B + q % B : (int64_t)i0 * B + q);
            if (k == 0 || k == nr - 1) atomicAdd(o, (OT)v);
            else *o = (OT)((double)*o + v);
        }
        __syncthreads();
    }
}

template <typename T, int B>
__global__ void k_phase2_prep_b(int64_t n, int32_t nN, const int32_t *perm, SrcSet src, const T *h,
                                const double *pibar, const int32_t *deg, double c, double *w2, double *xD) {
    const int64_t total = n * B;
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kBlock) {
        const int64_t v = idx / B;
        if (v < nN) {
            w2[idx] = c * (pibar[idx] + (double)h[idx]) / (double)deg[v];
        } else {
            xD[idx - (int64_t)nN * B] = h0_col<T>(src.s[idx % B], perm[v], n);
        }
    }
}

template <typename T, int B>
__device__ __forceinline__ double x_b(int64_t idx, int64_t nN, const T *h, const double *pibar, const double *xD) {
    const int64_t v = idx / B;
    return v < nN ? pibar[idx] + (double)h[idx] : xD[idx - nN * B];
}

template <typename T, int B>
__global__ __launch_bounds__(kBlock) void k_final_sum_b(int64_t n, int32_t nN, const T *h, const double *pibar,
                                                        const double *xD, double *part) {
    double s = 0.0, sn = 0.0;
    const int64_t total = n * B;
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kBlock) {
        s += x_b<T, B>(idx, nN, h, pibar, xD);
        if (idx / B < nN) sn += (double)h[idx];
    }
    __shared__ double sd[kBlock / W * B];
    const double rs = block_sum_cols<B>(s, sd);
    const double rn = block_sum_cols<B>(sn, sd);
    if (threadIdx.x < B) {
        part[threadIdx.x * gridDim.x + blockIdx.x] = rs;
        part[(B + threadIdx.x) * gridDim.x + blockIdx.x] = rn;
    }
}

template <int B>
__global__ __launch_bounds__(1024) void k_final_decide_b(CtlB *ctl, int nb, const double *part) {
    const int wv = threadIdx.x / W;
    for (int r = wv; r < 2 * B; r += blockDim.x / W) {
        double s = 0.0;
        for (int b = lane_id(); b < nb; b += W) s += part[(int64_t)r * nb + b];
        s = wave_sum(s);
        if (lane_id() == 0) {
            if (r < B) ctl->fin_sum[r] = s;
            else ctl->fin_sn[r - B] = s;
        }
    }
}

// out.p[j][original id] = x / sum_j for the columns in `mask`
template <typename T, int B>
__global__ void k_final_write_b(const CtlB *ctl, int64_t n, int32_t nN, const int32_t *perm, uint32_t mask,
                                OutSet out, const T *h, const double *pibar, const double *xD) {
    const int64_t total = n * B;
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kBlock) {
        const int jj = (int)(idx % B);
        if (!((mask >> jj) & 1u)) continue;
        const int64_t v = idx / B;
        out.p[jj][perm[v]] = x_b<T, B>(idx, nN, h, pibar, xD) / ctl->fin_sum[jj];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int B>
hipError_t launch_init_b(int64_t n, int32_t nN, const int32_t *perm, const SrcSet &src, uint32_t mask, T *h,
                         double *pibar, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_init_b<T, B>), dim3(grid_for(n * B, 4, 16384)), dim3(kBlock), 0, s, n, nN,
                       perm, src, mask, h, pibar);
    return hipGetLastError();
}

template <typename T, int B>
hipError_t launch_reserve_b(int t, CtlB *ctl, int32_t nN, T *h, T *w, double *pibar, const int32_t *deg,
                            const uint32_t *rp_nn, double c, double xi, int stop_l1, double tol, double pull_thr,
                            int force, unsigned long long pull_edges, double *part, hipStream_t s) {
    const int nb = grid_for((int64_t)nN * B, 4, kRedBlocks);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reserve_b<T, B>), dim3(nb), dim3(kBlock), 0, s, t, (const CtlB *)ctl, 0, nN,
                       h, w, pibar, deg, rp_nn, c, (T)xi, (const float *)nullptr, part);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_decide_b<B>), dim3(1), dim3(1024), 0, s, t, ctl, nb, (const double *)part,
                       c, stop_l1, tol, pull_thr, force, pull_edges);
    return hipGetLastError();
}

template <typename T, int B>
hipError_t launch_reserve_range_b(int t, CtlB *ctl, int32_t lo, int32_t hi, T *h, T *w, double *pibar,
                                  const int32_t *deg, const uint32_t *rp_nn, double c, double xi, const float *qle,
                                  int nb, double *part, hipStream_t s) {
    if (hi <= lo || nb < 1 || nb > kGroupBlocks || !qle) return hipErrorInvalidValue;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reserve_b<T, B>), dim3(nb), dim3(kBlock), 0, s, t, (const CtlB *)ctl, lo, hi,
                       h, w, pibar, deg, rp_nn, c, (T)xi, qle, part);
    return hipGetLastError();
}

template <int B>
hipError_t launch_decide_gs_b(int t, CtlB *ctl, int ngr, const GroupBlocks &gb, const double *part, double *sums,
                              double c, int stop_l1, double tol, double pull_thr, unsigned long long sweep_edges,
                              hipStream_t s) {
    if (ngr < 1 || ngr > kMaxGroups) return hipErrorInvalidValue;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rowsum_gs_b<B>), dim3(5 * B * ngr), dim3(kBlock), 0, s, t,
                       (const CtlB *)ctl, gb, part, sums);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_decide_gs_b<B>), dim3(1), dim3(kBlock), 0, s, t, ctl, ngr,
                       (const double *)sums, c, stop_l1, tol, pull_thr, sweep_edges);
    return hipGetLastError();
}

template <typename T, int B>
hipError_t launch_push_b(int t, const CtlB *ctl, const MPPlan &p, const T *w, T *h, int check_mode, hipStream_t s) {
    if (p.blocks == 0 || p.edges() == 0) return hipSuccess;
    auto kern = &k_push_b<T, B, kMPK>;
    static const int grid = resident_grid(kern);
    hipLaunchKernelGGL(kern, dim3(std::min(p.blocks, grid)), dim3(kBlock), 0, s, t, ctl, check_mode, p.rp, p.R, p.idx,
                       (const uint2 *)p.plan, p.items, p.blocks, w, h);
    return hipGetLastError();
}

template <typename WT, typename OT, int B>
hipError_t launch_pull_b(int t, const CtlB *ctl, const MPPlan &p, const WT *w, OT *out, int check_mode,
                         hipStream_t s) {
    if (p.blocks == 0 || p.edges() == 0) return hipSuccess;
    if (p.ipb != (kBlock / B) * kMPK) return hipErrorInvalidValue;  // the plan's tiles are the kernel's
    auto kern = &k_pull_b<WT, OT, B, kMPK>;
    static const int grid = resident_grid(kern);
    hipLaunchKernelGGL(kern, dim3(std::min(p.blocks, grid)), dim3(kBlock), 0, s, t, ctl, check_mode, p.rp, p.R, p.idx,
                       (const uint2 *)p.plan, p.items, p.blocks, p.rid, w, out);
    return hipGetLastError();
}

template <typename T, int B>
hipError_t launch_phase2_b(int64_t n, int32_t nN, const int32_t *perm, const SrcSet &src, const T *h,
                           const double *pibar, const int32_t *deg, double c, double *w2, double *xD,
                           const MPPlan &pull_nd, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_phase2_prep_b<T, B>), dim3(grid_for(n * B, 4, 16384)), dim3(kBlock), 0, s, n,
                       nN, perm, src, h, pibar, deg, c, w2, xD);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_pull_b<double, double, B>(-1, nullptr, pull_nd, w2, xD, 0, s);
}

template <typename T, int B>
hipError_t launch_final_b(CtlB *ctl, int64_t n, int32_t nN, const int32_t *perm, uint32_t mask, const OutSet &out,
                          const T *h, const double *pibar, const double *xD, double *part, hipStream_t s) {
    const int nb = grid_for(n * B, 4, kRedBlocks);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_final_sum_b<T, B>), dim3(nb), dim3(kBlock), 0, s, n, nN, h, pibar, xD, part);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_final_decide_b<B>), dim3(1), dim3(1024), 0, s, ctl, nb,
                       (const double *)part);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_final_write_b<T, B>), dim3(grid_for(n * B, 4, 16384)), dim3(kBlock), 0, s,
                       (const CtlB *)ctl, n, nN, perm, mask, out, h, pibar, xD);
    return hipGetLastError();
}

#define PRK_BATCH_INST(T, B)                                                                                         \
    template hipError_t launch_init_b<T, B>(int64_t, int32_t, const int32_t *, const SrcSet &, uint32_t, T *,       \
                                            double *, hipStream_t);                                                  \
    template hipError_t launch_reserve_b<T, B>(int, CtlB *, int32_t, T *, T *, double *, const int32_t *,           \
                                               const uint32_t *, double, double, int, double, double, int,          \
                                               unsigned long long, double *, hipStream_t);                          \
    template hipError_t launch_push_b<T, B>(int, const CtlB *, const MPPlan &, const T *, T *, int, hipStream_t);   \
    template hipError_t launch_pull_b<T, T, B>(int, const CtlB *, const MPPlan &, const T *, T *, int, hipStream_t); \
    template hipError_t launch_phase2_b<T, B>(int64_t, int32_t, const int32_t *, const SrcSet &, const T *,         \
                                              const double *, const int32_t *, double, double *, double *,          \
                                              const MPPlan &, hipStream_t);                                          \
    template hipError_t launch_final_b<T, B>(CtlB *, int64_t, int32_t, const int32_t *, uint32_t, const OutSet &,  \
                                             const T *, const double *, const double *, double *, hipStream_t);

PRK_BATCH_INST(float, 8)
PRK_BATCH_INST(double, 8)
PRK_BATCH_INST(float, 16)
PRK_BATCH_INST(double, 16)

#define PRK_BATCH_GS_INST(T, B)                                                                                     \
    template hipError_t launch_reserve_range_b<T, B>(int, CtlB *, int32_t, int32_t, T *, T *, double *,           \
                                                     const int32_t *, const uint32_t *, double, double,            \
                                                     const float *, int, double *, hipStream_t);
PRK_BATCH_GS_INST(float, 8)
PRK_BATCH_GS_INST(double, 8)
PRK_BATCH_GS_INST(float, 16)
PRK_BATCH_GS_INST(double, 16)
template hipError_t launch_decide_gs_b<8>(int, CtlB *, int, const GroupBlocks &, const double *, double *, double,
                                          int, double, double, unsigned long long, hipStream_t);
template hipError_t launch_decide_gs_b<16>(int, CtlB *, int, const GroupBlocks &, const double *, double *, double,
                                           int, double, double, unsigned long long, hipStream_t);

}  // namespace prk
