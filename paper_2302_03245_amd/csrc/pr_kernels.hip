// pr_kernels.hip -- gfx950 kernels of libpr.so.
//
// The path is sparse and memory bound (one multiply-add and one scattered add
// per edge), so nothing here uses the matrix cores.  Work is organised for
// 64-wide waves: wave ballots for compaction and row splitting, LDS-staged
// merge-path tiles for edge streaming, FP64 block reductions finished by the
// last workgroup of a launch.
#include <hip/hip_ext.h>

#include "pr_device.h"

#include <limits.h>

#include <algorithm>

namespace prk {

namespace {

// ------------------------------------------------------------------------
// graph preparation
// ------------------------------------------------------------------------
__global__ void k_check_cols(const int32_t *col, int64_t m, int64_t n, unsigned int *bad) {
    unsigned int b = 0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock) {
        int32_t c = col[e];
        b |= (c < 0 || (int64_t)c >= n);
    }
    if (__any(b) && lane_id() == 0) atomicOr(bad, 1u);
}

__global__ void k_degree_class(const int64_t *rp, int64_t n, uint32_t *isN) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        isN[i] = rp[i + 1] > rp[i] ? 1u : 0u;
}

__global__ void k_indegree(const int32_t *col, int64_t m, uint32_t *indeg) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
        atomicAdd(indeg + col[e], 1u);
}

// exclusive scan, 16 elements per thread, 4096 per block
constexpr int kScanPer = 16;
constexpr int kScanTile = kBlock * kScanPer;

__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t s_w[kBlock / W];
    uint32_t inc = wave_incl_scan(v);
    if (lane_id() == W - 1) s_w[threadIdx.x / W] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / W; ++k) {
        uint32_t s = s_w[k];
        if (k < (int)(threadIdx.x / W)) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void k_scan_partial(const uint32_t *in, int64_t n, uint32_t *partial) {
    int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanPer;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) s += in[base + k];
    __shared__ uint32_t sb[kBlock / W];
    uint32_t tot = block_sum(s, sb);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_scan_top(uint32_t *partial, int64_t nb) {
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? partial[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
    }
}

__global__ void k_scan_final(const uint32_t *in, uint32_t *out, int64_t n, const uint32_t *partial) {
    int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kScanPer;
    uint32_t vals[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        vals[k] = base + k < n ? in[base + k] : 0u;
        s += vals[k];
    }
    uint32_t tot;
    uint32_t run = partial[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += vals[k];
    }
    if (base <= n - 1 && n - 1 < base + kScanPer) out[n] = run;  // the thread holding the last element
}

__global__ void k_relabel(const uint32_t *isN, const uint32_t *rankN, int64_t n, int32_t nN, int32_t *newid,
                          int32_t *perm) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        uint32_t r = rankN[i];
        int32_t id = isN[i] ? (int32_t)r : (int32_t)(nN + (i - (int64_t)r));
        newid[i] = id;
        perm[id] = (int32_t)i;
    }
}

// one wave per non-dangling row: number of targets that are non-dangling
__global__ void k_count_nn(const int64_t *rp, const int32_t *col, const uint32_t *isN, const int32_t *perm,
                           int32_t nN, uint32_t *cnt_nn, uint32_t *cnt_nd, int32_t *deg) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t k = wave; k < nN; k += nwaves) {
        int32_t i = perm[k];
        int64_t lo = rp[i], hi = rp[i + 1];
        uint32_t c = 0;
        for (int64_t e = lo + lane_id(); e - lane_id() < hi; e += W) {
            bool t = e < hi && isN[col[e]];
            c += (uint32_t)__popcll(__ballot(t));
        }
        if (lane_id() == 0) {
            cnt_nn[k] = c;
            cnt_nd[k] = (uint32_t)(hi - lo) - c;
            deg[k] = (int32_t)(hi - lo);
        }
    }
}

// one wave per non-dangling row: stable split of the row into N targets and D targets (new ids)
__global__ void k_split_rows(const int64_t *rp, const int32_t *col, const uint32_t *isN, const int32_t *newid,
                             const int32_t *perm, int32_t nN, const uint32_t *rp_nn, int32_t *col_nn,
                             const uint32_t *rp_nd, int32_t *col_nd) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    const unsigned long long lt = (1ull << lane_id()) - 1ull;
    for (int64_t k = wave; k < nN; k += nwaves) {
        int32_t i = perm[k];
        int64_t lo = rp[i], hi = rp[i + 1];
        uint32_t on = rp_nn[k], od = rp_nd[k];
        for (int64_t e = lo + lane_id(); e - lane_id() < hi; e += W) {
            bool valid = e < hi;
            int32_t t = valid ? col[e] : 0;
            bool tn = valid && isN[t];
            unsigned long long mn = __ballot(tn), md = __ballot(valid && !tn);
            if (tn) col_nn[on + __popcll(mn & lt)] = newid[t];
            else if (valid) col_nd[od + __popcll(md & lt)] = newid[t];
            on += (uint32_t)__popcll(mn);
            od += (uint32_t)__popcll(md);
        }
    }
}

__global__ void k_permute_u32(const uint32_t *in_old, const int32_t *perm, int64_t n, uint32_t *out_new) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        out_new[k] = in_old[perm[k]];
}

// one wave per source row: append the source to each target's in-list
__global__ void k_fill_csc(const uint32_t *rp, const int32_t *col, int32_t R, uint32_t *cursor, int32_t *in_src) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t k = wave; k < R; k += nwaves) {
        uint32_t lo = rp[k], hi = rp[k + 1];
        for (uint32_t e = lo + lane_id(); e < hi; e += W) {
            uint32_t pos = atomicAdd(cursor + col[e], 1u);
            in_src[pos] = (int32_t)k;
        }
    }
}

__global__ void k_count_zero(const uint32_t *a, int64_t n, unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        c += a[i] == 0u;
    __shared__ unsigned long long sb[kBlock / W];
    c = block_sum(c, sb);
    if (threadIdx.x == 0 && c) atomic_add_u64(out, c);
}

// ---- unreferenced depth of the non-dangling vertices (Kahn rounds on the N -> N edges)
// depth(v) = 0 without non-dangling in-neighbours, else 1 + max depth of them;
// vertices on or below a cycle keep kDepthInf.  After sweep depth(v) no mass can
// reach v again, so from sweep depth(v) + 1 on its push weight is zero.

// append the lanes' items with one atomic per wave
__device__ __forceinline__ void wave_append(bool take, int32_t v, int32_t *q, uint32_t *count) {
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, W);
    if (take) q[base + __popcll(mask & ((1ull << lane_id()) - 1ull))] = v;
}

__global__ void k_depth_init(int32_t nN, const uint32_t *in_ptr, uint32_t *rem, int32_t *depth, int32_t *q,
                             uint32_t *qcount) {
    for (int64_t base = blockIdx.x * (int64_t)kBlock; base < nN; base += (int64_t)gridDim.x * kBlock) {
        const int64_t v = base + threadIdx.x;
        bool zero = false;
        if (v < nN) {
            const uint32_t r = in_ptr[v + 1] - in_ptr[v];
            rem[v] = r;
            depth[v] = r == 0 ? 0 : kDepthInf;
            zero = r == 0;
        }
        wave_append(zero, (int32_t)v, q, qcount);
    }
}

// one wave per vertex of the current round: release its out-neighbours
__global__ void k_depth_step(const int32_t *q, uint32_t qsize, const uint32_t *rp_nn, const int32_t *col_nn,
                             uint32_t *rem, int32_t *depth, int32_t round, int32_t *next, uint32_t *ncount) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t k = wave; k < qsize; k += nwaves) {
        const int32_t v = q[k];
        const uint32_t lo = rp_nn[v], hi = rp_nn[v + 1];
        for (uint32_t e = lo + lane_id(); e - lane_id() < hi; e += W) {
            bool done = false;
            int32_t u = 0;
            if (e < hi) {
                u = col_nn[e];
                if (atomicSub(rem + u, 1u) == 1u) {
                    depth[u] = round + 1;
                    done = true;
                }
            }
            wave_append(done, u, next, ncount);
        }
    }
}

// one wave per target row: number of in-edges whose source depth is >= t0
// (also restricted to sources in [slo, shi): the in-lists of one source group)
__global__ void k_live_count(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                             int32_t t0, int32_t slo, int32_t shi, const uint8_t *grp, int32_t q, uint32_t *cnt) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t r = wave; r < R; r += nwaves) {
        const uint32_t lo = in_ptr[r], hi = in_ptr[r + 1];
        uint32_t c = 0;
        for (uint32_t e = lo + lane_id(); e - lane_id() < hi; e += W) {
            const int32_t u = e < hi ? in_src[e] : 0;
            const bool live = e < hi && u >= slo && u < shi && depth[u] >= t0 && (!grp || grp[u] == q);
            c += (uint32_t)__popcll(__ballot(live));
        }
        if (lane_id() == 0) cnt[r] = c;
    }
}

// one wave per target row: copy the live in-edges, order kept
__global__ void k_live_fill(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                            int32_t t0, int32_t slo, int32_t shi, const uint8_t *grp, int32_t q,
                            const uint32_t *out_ptr, int32_t *out_src) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    const unsigned long long lt = (1ull << lane_id()) - 1ull;
    for (int64_t r = wave; r < R; r += nwaves) {
        const uint32_t lo = in_ptr[r], hi = in_ptr[r + 1];
        uint32_t o = out_ptr[r];
        for (uint32_t e = lo + lane_id(); e - lane_id() < hi; e += W) {
            const int32_t u = e < hi ? in_src[e] : 0;
            const bool live = e < hi && u >= slo && u < shi && depth[u] >= t0 && (!grp || grp[u] == q);
            const unsigned long long mk = __ballot(live);
            if (live) out_src[o + __popcll(mk & lt)] = u;
            o += (uint32_t)__popcll(mk);
        }
    }
}

// rows with an edge in a vertex group's in-lists (see launch_row_flags)
__global__ void k_row_flags(int32_t R, const uint32_t *cnt, uint32_t *flag) {
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < R; r += (int64_t)gridDim.x * kBlock)
        flag[r] = cnt[r] > 0 ? 1u : 0u;
}

__global__ void k_row_fill(int32_t R, const uint32_t *cnt, const uint32_t *pos, const uint32_t *off, int32_t *rid,
                           uint32_t *rp) {
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r <= R; r += (int64_t)gridDim.x * kBlock) {
        if (r == R) {
            rp[pos[R]] = off[R];
        } else if (cnt[r] > 0) {
            rid[pos[r]] = (int32_t)r;
            rp[pos[r]] = off[r];
        }
    }
}

// merge-path split points: plan[b] = (rows finished before diagonal d, edge at d)
__global__ void k_plan(const uint32_t *rp, int32_t R, uint32_t items, int32_t ipb, int32_t blocks, uint2 *plan) {
    const uint32_t rp0 = rp[0];
    for (int64_t b = blockIdx.x * (int64_t)kBlock + threadIdx.x; b <= blocks; b += (int64_t)gridDim.x * kBlock) {
        uint64_t dd = (uint64_t)b * (uint64_t)ipb;
        uint32_t d = dd < items ? (uint32_t)dd : items;
        int32_t lo = 0, hi = R;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (rp[mid + 1] - rp0 + (uint32_t)mid < d) lo = mid + 1;
            else hi = mid;
        }
        plan[b] = make_uint2((uint32_t)lo, rp0 + d - (uint32_t)lo);
    }
}

// ------------------------------------------------------------------------
// forward-push sweep kernels
// ------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ double h0_of(const InitArgs &a, int64_t i) {
    if (a.source >= 0) return a.perm[i] == a.source ? (double)a.n : 0.0;
    if (a.uniform) return 1.0;
    return (double)a.n * a.p[a.perm[i]] * a.pscale;
}

template <typename T>
__global__ void k_init_ifp(InitArgs a, T *h, double *pibar) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        h[i] = (T)h0_of<T>(a, i);
        if (i < a.nN) pibar[i] = 0.0;
    }
}

// Sums of N values over the workgroup in one pass (results in thread 0, each
// summed in the same order as block_sum); sbuf holds N * kBlock / W entries.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double *sbuf) {
    constexpr int NW = kBlock / W;
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
    if (lane_id() == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) sbuf[q * NW + threadIdx.x / W] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < NW; ++k) r += sbuf[q * NW + k];
            v[q] = r;
        }
    }
}

// Sums of N partial arrays of nb <= kRedBlocks entries each (array q at part + q nb)
// in one pass: every load issues before any add, each thread adds its entries in
// index order, then one workgroup reduction -- the same sums, in the same order, as
// N calls of reduce_partials.  Results in thread 0; sbuf holds N * kBlock / W entries.
template <int N>
__device__ __forceinline__ void reduce_partials_n(const double *part, int nb, double (&v)[N], double *sbuf) {
    constexpr int R = kRedBlocks / kBlock;
    static_assert(kRedBlocks % kBlock == 0, "partials");
    double x[N][R];
#pragma unroll
    for (int q = 0; q < N; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int b = threadIdx.x + r * kBlock;
            x[q][r] = b < nb ? part[(size_t)q * nb + b] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) acc += x[q][r];
        v[q] = acc;
    }
    block_sum_n(v, sbuf);
}

// Reserve step of one sweep (the body of the calculation threads' loop):
// every non-dangling i with h_i > xi moves its residual v into pibar_i and
// publishes its push weight w_i = c v / deg(i); others publish 0.  Per
// workgroup partial sums: residual left on inactive vertices, mass this
// sweep sends to non-dangling vertices, growth of the total mass, active
// vertices and their valid edges.  The kernel is bound by the latency of its
// loads when the grid holds about one vertex per thread (the small vertex
// groups of ordered sweeps) and when most vertices are active (a dense
// frontier: ctl->use_pull, set by the last decision): then a vertex's degree,
// row offsets and pibar are loaded together with its residual, two vertices
// per iteration, instead of after the test.  Sums run in the same order either way.
// With error weights (ew.g non-null) the residual left and the mass sent to N are
// weighted by g and q (the stop rule's weighted bound).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reserve(int t, const Ctl *ctl, int32_t lo, int32_t hi, T *h, T *w,
                                                    double *pibar, const int32_t *deg, const uint32_t *rp_nn,
                                                    double c, T xi, int ifp2, ErrWeights ew, double *part) {
    if (t > ctl->stop_after) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // uniform over the grid
    const bool eager = (int64_t)(hi - lo) <= stride || ctl->use_pull != 0;
    double inact = 0.0, pred = 0.0, sxinc = 0.0;
    unsigned long long cnt = 0, edges = 0;
    // one vertex whose inputs are loaded (dg, r0, r1, pb are read only when active)
    auto take = [&](int64_t i, T hv, int32_t dg, uint32_t r0, uint32_t r1, double pb) {
        // |h_i| > xi: residuals are non-negative except after a warm start
        if (hv > xi || hv < -xi) {
            const uint32_t dnn = r1 - r0;
            const double v = (double)hv;
            pibar[i] = pb + v;
            h[i] = (T)0;
            w[i] = (T)(c * v / (double)dg);
            const double fN = (double)dnn / (double)dg;
            pred += fabs(v) * (ew.q ? (double)ew.q[i] : fN);
            sxinc += ifp2 ? v * fN : v;
            cnt += 1;
            edges += ifp2 ? dnn : (uint32_t)dg;
        } else {
            w[i] = (T)0;
            inact += fabs((double)hv) * (ew.g ? (double)ew.g[i] : 1.0);
        }
    };
    int64_t i = lo + blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (eager) {
        for (; i < hi; i += 2 * stride) {
            const int64_t i2 = i + stride;
            const bool two = i2 < hi;
            const T hv = h[i];
            const int32_t dg = deg[i];
            const uint32_t r0 = rp_nn[i], r1 = rp_nn[i + 1];
            const double pb = pibar[i];
            T hv2 = (T)0;
            int32_t dg2 = 1;
            uint32_t s0 = 0, s1 = 0;
            double pb2 = 0.0;
            if (two) {
                hv2 = h[i2];
                dg2 = deg[i2];
                s0 = rp_nn[i2];
                s1 = rp_nn[i2 + 1];
                pb2 = pibar[i2];
            }
            take(i, hv, dg, r0, r1, pb);
            if (two) take(i2, hv2, dg2, s0, s1, pb2);
        }
    } else {
        for (; i < hi; i += stride) {
            const T hv = h[i];
            if (hv > xi || hv < -xi) take(i, hv, deg[i], rp_nn[i], rp_nn[i + 1], pibar[i]);
            else take(i, hv, 0, 0, 0, 0.0);
        }
    }
    __shared__ double sd[5 * (kBlock / W)];
    double v[5] = {inact, pred, sxinc, (double)cnt, (double)edges};
    block_sum_n(v, sd);
    if (threadIdx.x == 0) {
        const int nb = gridDim.x, b = blockIdx.x;
#pragma unroll
        for (int q = 0; q < 5; ++q) part[q * nb + b] = v[q];
    }
}

// Certified L1 bound on the normalised result from the residual sum sn (of |h| over
// the non-dangling vertices) and the total mass sx, k = 2c / (1 - c).  Non-negative
// residuals: the exact unnormalised vector is at least the estimate, so k sn / sx.
// Signed residuals (warm start): the estimate may exceed it, and its mass is only
// known within E = (k / 2) sn, so k sn / (sx - E) (the final figure of the solve also
// carries the estimate's negative part).
__device__ __forceinline__ double l1_bound_of(double k, double sn, double sx, int signed_res) {
    if (!signed_res) return k * sn / sx;
    const double den = sx - 0.5 * k * sn;
    return den > 0.0 ? k * sn / den : INFINITY;
}

// Residual left on the non-dangling vertices after an ordered sweep (per
// workgroup partials): S_N of the stop rule, summed directly because mass a
// group pushes may already have been taken by a later group of the same sweep.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sum_h(int t, const Ctl *ctl, int32_t nN, const T *h, const float *g,
                                                  double *part) {
    if (t > ctl->stop_after) return;
    // eight loads in flight per thread, added in index order (weighted by g when given)
    constexpr int U = 8;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double s = 0.0;
    for (int64_t i0 = blockIdx.x * (int64_t)kBlock + threadIdx.x; i0 < nN; i0 += U * stride) {
        T x[U];
        float gv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            x[u] = i < nN ? h[i] : (T)0;
            gv[u] = (g && i < nN) ? g[i] : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += fabs((double)x[u]) * (double)gv[u];
    }
    __shared__ double sd[kBlock / W];
    s = block_sum(s, sd);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Management step of an ordered sweep (one workgroup), after all groups have
// reserved and gathered: the growth of the total mass and the work from the
// groups' reserve partials (group g: gb.nb[g] workgroups, 5 sums each), S_N
// from k_sum_h; stop when nothing was above the threshold or the certified
// bound is met.  One pass over all partials, then one workgroup reduction of
// the four sums.
__global__ __launch_bounds__(kBlock) void k_decide_gs(int t, Ctl *ctl, Trace *tr, int ng, GroupBlocks gb,
                                                      const double *part, int nbs, const double *part_s, double c,
                                                      double kb, int stop_l1, double tol,
                                                      unsigned long long pull_thr, unsigned long long pull_edges,
                                                      int bookkeep) {
    if (t > ctl->stop_after) return;
    // a group has at most kGroupRounds * kBlock reserve workgroups (and k_sum_h at
    // most as many): every partial of a group, or of S_N, is loaded before any is added
    constexpr int kGroupRounds = 4;
    static_assert(kGroupBlocks <= kGroupRounds * kBlock && kRedBlocks <= kGroupRounds * kBlock, "partials");
    __shared__ double sd[4 * (kBlock / W)];
    // bookkeep: S_N from the reserves' own sums, each group's residual left behind (part 0)
    // plus c times its pushed mass weighted by the part that stays residual to the end of
    // the sweep (part 1); else from k_sum_h's direct sum (part_s)
    double a_sx = 0.0, a_cd = 0.0, a_ed = 0.0, sn = 0.0;
    for (int g = 0; g < ng; ++g) {
        const double *pg = part + (size_t)g * 5 * gb.stride;
        const int nb = gb.nb[g];
        double x[kGroupRounds][5];
#pragma unroll
        for (int r = 0; r < kGroupRounds; ++r) {
            const int b = threadIdx.x + r * kBlock;
            const bool in = b < nb;
            x[r][0] = in ? pg[2 * nb + b] : 0.0;
            x[r][1] = in ? pg[3 * nb + b] : 0.0;
            x[r][2] = in ? pg[4 * nb + b] : 0.0;
            x[r][3] = in && bookkeep ? pg[b] : 0.0;
            x[r][4] = in && bookkeep ? pg[nb + b] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kGroupRounds; ++r) {
            if (threadIdx.x + r * kBlock < nb) {
                a_sx += x[r][0];
                a_cd += x[r][1];
                a_ed += x[r][2];
                sn += x[r][3] + c * x[r][4];
            }
        }
    }
    {
        double x[kGroupRounds];
#pragma unroll
        for (int r = 0; r < kGroupRounds; ++r) {
            const int b = threadIdx.x + r * kBlock;
            x[r] = b < nbs ? part_s[b] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kGroupRounds; ++r)
            if (threadIdx.x + r * kBlock < nbs) sn += x[r];
    }
    double v[4] = {a_sx, a_cd, a_ed, sn};
    block_sum_n(v, sd);
    if (threadIdx.x != 0) return;
    a_sx = v[0];
    a_cd = v[1];
    a_ed = v[2];
    sn = v[3];
    const unsigned long long a_c = (unsigned long long)a_cd, a_e = (unsigned long long)a_ed;
    const double k = kb;
    const double sx = ctl->sx + c * a_sx;
    const double bound = l1_bound_of(k, sn, sx, ctl->signed_res);
    ctl->sx = sx;
    ctl->sn_last = sn;
    ctl->last_edges = a_e;
    ctl->last_bound = bound;
    if (a_c == 0) {
        ctl->stop_after = t - 1;  // nothing moved in this sweep
    } else {
        ctl->sweeps = t + 1;
        ctl->tot_pushes += a_c;
        ctl->tot_edges += a_e;
        ctl->use_pull = a_e >= pull_thr ? 1 : 0;  // would a synchronous sweep gather (is the frontier dense)
        ctl->pull_sweeps += 1;
        ctl->tot_traversed += pull_edges;
        if (stop_l1 && bound <= tol) ctl->stop_after = t;
    }
    if (t < kMaxTrace) {
        tr->cnt[t] = a_c | (a_c ? (1ull << 63) : 0ull);
        tr->edges[t] = a_e;
        tr->sn[t] = sn;
        tr->bound[t] = bound;
    }
}

// Management step of one sweep (one workgroup): sums the reserve partials and
// decides -- stop (no vertex above the threshold, or the certified L1 bound
// after this sweep's pushes is met), and push or pull for the scatter.
__global__ __launch_bounds__(kBlock) void k_decide_ifp(int t, Ctl *ctl, Trace *tr, int nb, const double *part,
                                                       double c, double kb, int stop_l1, double tol,
                                                       unsigned long long pull_thr, int force,
                                                       unsigned long long pull_edges) {
    if (t > ctl->stop_after) return;
    __shared__ double sd[5 * (kBlock / W)];
    double v[5];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x != 0) return;
    const double a_in = v[0], a_pr = v[1], a_sx = v[2], a_cd = v[3], a_ed = v[4];
    const unsigned long long a_c = (unsigned long long)a_cd, a_e = (unsigned long long)a_ed;
    const double k = kb;
    if (a_c == 0) {
        // nothing above the threshold: the state is unchanged, stop before this sweep's scatter
        ctl->stop_after = t - 1;
        ctl->sn_last = a_in;
        ctl->last_edges = 0;
        ctl->last_bound = l1_bound_of(k, a_in, ctl->sx, ctl->signed_res);
        if (t < kMaxTrace) {
            tr->cnt[t] = 0;
            tr->edges[t] = 0;
            tr->sn[t] = a_in;
            tr->bound[t] = ctl->last_bound;
        }
        return;
    }
    const double sn = a_in + c * a_pr;
    const double sx = ctl->sx + c * a_sx;
    const double bound = l1_bound_of(k, sn, sx, ctl->signed_res);
    ctl->sx = sx;
    ctl->sn_last = sn;
    ctl->last_edges = a_e;
    ctl->sweeps = t + 1;
    ctl->tot_pushes += a_c;
    ctl->tot_edges += a_e;
    const int pull = force == 1 ? 0 : (force == 2 ? 1 : (a_e >= pull_thr ? 1 : 0));
    ctl->use_pull = pull;
    ctl->pull_sweeps += pull;
    ctl->tot_traversed += pull ? pull_edges : a_e;
    ctl->last_bound = bound;
    if (stop_l1 && bound <= tol) ctl->stop_after = t;
    if (t < kMaxTrace) {
        tr->cnt[t] = a_c | ((unsigned long long)pull << 63);
        tr->edges[t] = a_e;
        tr->sn[t] = sn;
        tr->bound[t] = bound;
    }
}

// ------------------------------------------------------------------------
// list sweeps: the frontier {i in N : h_i > xi} of Algorithms 2 and 3 kept as a
// compacted list of vertex ids, so a sparse sweep costs O(frontier + its edges)
// instead of a pass over every non-dangling vertex.  A list is written with one
// counter atomic per wave: the wave's ballot of set lanes gives the count, and each
// lane's rank among them (mbcnt over the ballot) its offset.  The scatter uses
// returning atomics: the one add that lifts h_j from <= xi to > xi appends j to the
// next sweep's list (the residual only grows during a scatter, so exactly one add
// crosses), which keeps every vertex above the threshold listed once.
// ------------------------------------------------------------------------

// Slot of each lane with pred set in a list counted by *cnt (one atomic per wave); the
// return value is meaningful only where pred is set.  Call with the whole wave active.
__device__ __forceinline__ uint32_t wave_slot(bool pred, uint32_t *cnt) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return 0u;
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0u;
    if (lane_id() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader, W);
    return base + rank;
}

// Frontier list from the residuals (the start of a run of list sweeps): every
// non-dangling i with h_i > xi, into f (slot `slot` of the counters, zero on entry).
// Also the residual on the non-dangling vertices (per workgroup partials), from which
// list sweeps carry it forward.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_compact(Ctl *ctl, int slot, int32_t nN, const T *h, T xi, int32_t *f,
                                                    const int32_t *deg, const uint32_t *rp_nn, int ifp2,
                                                    const float *g, double *part) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double sn = 0.0;
    unsigned long long ve = 0;
    // the trip count is uniform over a wave (its lanes share `base`)
    for (int64_t base = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~(W - 1)); base < nN; base += stride) {
        const int64_t i = base + lane_id();
        const T hv = i < nN ? h[i] : (T)0;
        sn += (double)hv * ((g && i < nN) ? (double)g[i] : 1.0);
        const bool act = hv > xi;
        const uint32_t q = wave_slot(act, &ctl->fcnt[slot]);
        if (act) {
            f[q] = (int32_t)i;
            ve += ifp2 ? (unsigned long long)(rp_nn[i + 1] - rp_nn[i]) : (unsigned long long)deg[i];
        }
    }
    ve = wave_sum(ve);
    if (lane_id() == 0 && ve) atomic_add_u64(&ctl->fedges[slot], ve);
    __shared__ double sd[kBlock / W];
    sn = block_sum(sn, sd);
    if (threadIdx.x == 0) part[blockIdx.x] = sn;
}

__global__ __launch_bounds__(kBlock) void k_list_start(Ctl *ctl, int nb, const double *part) {
    __shared__ double sd[kBlock / W];
    const double sn = reduce_partials(part, nb, sd);
    if (threadIdx.x == 0) ctl->sn_last = sn;
}

// Reserve step of list sweep t over the frontier list of slot t & 1: each listed
// vertex moves its residual v into pibar_i and becomes scatter work with weight
// c v / deg(i) -- one lane item if it has at most kLaneEdges valid out-edges, else
// one wave item per chunk of kChunkEdges.  Partial sums per workgroup: mass taken,
// mass sent to non-dangling vertices, growth of the total mass, active vertices and
// their valid edges.  Also clears the counters the scatter of this sweep fills.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reserve_list(int t, Ctl *ctl, ListBufs<T> lb, T *h, double *pibar,
                                                         const int32_t *deg, const uint32_t *rp_nn, double c, T xi,
                                                         int ifp2, ErrWeights ew, double *part) {
    if (t > ctl->stop_after) return;
    const int b = t & 1;
    const uint32_t nf = ctl->fcnt[b];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->fcnt[b ^ 1] = 0u;  // next frontier (filled by this sweep's scatter)
        ctl->fedges[b ^ 1] = 0ull;
        ctl->lcnt[b ^ 1] = 0u;  // work lists of the next sweep
        ctl->wcnt[b ^ 1] = 0u;
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double taken = 0.0, pred = 0.0, sxinc = 0.0;
    unsigned long long cnt = 0, edges = 0;
    for (int64_t base = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~(W - 1)); base < (int64_t)nf; base += stride) {
        const int64_t q = base + lane_id();
        bool lane_item = false;
        int32_t i = 0;
        T wt = (T)0;
        uint32_t dv = 0;
        if (q < (int64_t)nf) {
            i = lb.f[b][q];
            const T hv = h[i];
            if (hv > xi) {
                const int32_t dg = deg[i];
                const uint32_t dnn = rp_nn[i + 1] - rp_nn[i];
                const double v = (double)hv;
                pibar[i] += v;
                h[i] = (T)0;
                wt = (T)(c * v / (double)dg);
                const double fN = (double)dnn / (double)dg;
                taken += v * (ew.g ? (double)ew.g[i] : 1.0);
                pred += v * (ew.q ? (double)ew.q[i] : fN);
                sxinc += ifp2 ? v * fN : v;
                dv = ifp2 ? dnn : (uint32_t)dg;
                cnt += 1;
                edges += dv;
                lane_item = dv > 0 && dv <= (uint32_t)kLaneEdges;
            }
        }
        const uint32_t ql = wave_slot(lane_item, &ctl->lcnt[b]);
        if (lane_item) {
            lb.lane_v[ql] = i;
            lb.lane_w[ql] = wt;
        }
        if (dv > (uint32_t)kLaneEdges) {  // long rows are rare: one atomic per row
            const uint32_t nch = (dv + kChunkEdges - 1) / kChunkEdges;
            const uint32_t q0 = atomicAdd(&ctl->wcnt[b], nch);
            for (uint32_t k = 0; k < nch; ++k) {
                lb.wave_v[q0 + k] = i;
                lb.wave_c[q0 + k] = (int32_t)k;
                lb.wave_w[q0 + k] = wt;
            }
        }
    }
    __shared__ double sd[5 * (kBlock / W)];
    double v[5] = {taken, pred, sxinc, (double)cnt, (double)edges};
    block_sum_n(v, sd);
    if (threadIdx.x == 0) {
        const int nb = gridDim.x, bb = blockIdx.x;
#pragma unroll
        for (int q = 0; q < 5; ++q) part[q * nb + bb] = v[q];
    }
}

// Management step of a list sweep: the residual left on N follows from the previous
// decision's sum (residuals are non-negative and only listed vertices were taken);
// otherwise as the synchronous sweep's decision.  List sweeps always scatter.
__global__ __launch_bounds__(kBlock) void k_decide_list(int t, Ctl *ctl, Trace *tr, int nb, const double *part,
                                                        double c, double kb, int stop_l1, double tol) {
    if (t > ctl->stop_after) return;
    __shared__ double sd[5 * (kBlock / W)];
    double v[5];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x != 0) return;
    const double taken = v[0], a_pr = v[1], a_sx = v[2];
    const unsigned long long a_c = (unsigned long long)v[3], a_e = (unsigned long long)v[4];
    const double k = kb;
    if (a_c == 0) {
        ctl->stop_after = t - 1;
        ctl->last_bound = l1_bound_of(k, ctl->sn_last, ctl->sx, 0);
        ctl->last_edges = 0;
        if (t < kMaxTrace) {
            tr->cnt[t] = 0;
            tr->edges[t] = 0;
            tr->sn[t] = ctl->sn_last;
            tr->bound[t] = ctl->last_bound;
        }
        return;
    }
    const double sn = fmax(ctl->sn_last - taken, 0.0) + c * a_pr;
    const double sx = ctl->sx + c * a_sx;
    const double bound = l1_bound_of(k, sn, sx, 0);
    ctl->sx = sx;
    ctl->sn_last = sn;
    ctl->last_edges = a_e;
    ctl->sweeps = t + 1;
    ctl->tot_pushes += a_c;
    ctl->tot_edges += a_e;
    ctl->use_pull = 0;
    ctl->tot_traversed += a_e;
    ctl->last_bound = bound;
    if (stop_l1 && bound <= tol) ctl->stop_after = t;
    if (t < kMaxTrace) {
        tr->cnt[t] = a_c;
        tr->edges[t] = a_e;
        tr->sn[t] = sn;
        tr->bound[t] = bound;
    }
}

// Scatter step of list sweep t: lane items walk their few edges one lane each, wave
// items one chunk per wave with the lanes on consecutive edges.  Every add returns the
// old residual; a non-dangling target crossing xi is appended to the next frontier.
// Edge k of row i: its non-dangling targets first, then (IFP1) those in the deferred region.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_push_list(int t, Ctl *ctl, ListBufs<T> lb, T *h, const int32_t *deg,
                                                      const uint32_t *rp_nn, const int32_t *col_nn,
                                                      const uint32_t *rp_nd, const int32_t *col_nd, T xi, int ifp2) {
    if (t > ctl->stop_after) return;
    const int b = t & 1;
    const uint32_t nl = ctl->lcnt[b], nw = ctl->wcnt[b];
    uint32_t *fc = &ctl->fcnt[b ^ 1];
    int32_t *fo = lb.f[b ^ 1];
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    unsigned long long ve = 0;  // valid out-edges of the vertices this thread appended
    auto valid_edges = [&](int32_t j) -> unsigned long long {
        return ifp2 ? (unsigned long long)(rp_nn[j + 1] - rp_nn[j]) : (unsigned long long)deg[j];
    };
    for (int64_t base = blockIdx.x * (int64_t)kBlock + (threadIdx.x & ~(W - 1)); base < (int64_t)nl; base += stride) {
        const int64_t q = base + lane_id();
        int32_t i = 0;
        T wt = (T)0;
        uint32_t r0 = 0, dnn = 0, d0 = 0, dv = 0;
        if (q < (int64_t)nl) {
            i = lb.lane_v[q];
            wt = lb.lane_w[q];
            r0 = rp_nn[i];
            dnn = rp_nn[i + 1] - r0;
            dv = dnn;
            if (!ifp2) {
                d0 = rp_nd[i];
                dv += rp_nd[i + 1] - d0;
            }
        }
        for (uint32_t k = 0; __ballot(k < dv) != 0ull; ++k) {  // uniform: until every lane's row is done
            bool cross = false;
            int32_t j = 0;
            if (k < dv) {
                j = k < dnn ? col_nn[r0 + k] : col_nd[d0 + (k - dnn)];
                const T old = atomicAdd(h + j, wt);
                cross = k < dnn && !(old > xi) && (T)(old + wt) > xi;
            }
            const uint32_t qf = wave_slot(cross, fc);
            if (cross) {
                fo[qf] = j;
                ve += valid_edges(j);
            }
        }
    }
    const int64_t nwaves = stride / W;
    for (int64_t q = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W; q < (int64_t)nw; q += nwaves) {
        const int32_t i = lb.wave_v[q];
        const T wt = lb.wave_w[q];
        const uint32_t r0 = rp_nn[i], dnn = rp_nn[i + 1] - r0;
        uint32_t d0 = 0, dv = dnn;
        if (!ifp2) {
            d0 = rp_nd[i];
            dv += rp_nd[i + 1] - d0;
        }
        const uint32_t k0 = (uint32_t)lb.wave_c[q] * kChunkEdges;
        const uint32_t k1 = min(dv, k0 + (uint32_t)kChunkEdges);
        for (uint32_t kb = k0; kb < k1; kb += W) {
            const uint32_t k = kb + lane_id();
            bool cross = false;
            int32_t j = 0;
            if (k < k1) {
                j = k < dnn ? col_nn[r0 + k] : col_nd[d0 + (k - dnn)];
                const T old = atomicAdd(h + j, wt);
                cross = k < dnn && !(old > xi) && (T)(old + wt) > xi;
            }
            const uint32_t qf = wave_slot(cross, fc);
            if (cross) {
                fo[qf] = j;
                ve += valid_edges(j);
            }
        }
    }
    ve = wave_sum(ve);
    if (lane_id() == 0 && ve) atomic_add_u64(&ctl->fedges[b ^ 1], ve);
}

// graph-set sweeps: a tile whose rows all belong to graphs that stopped before
// sweep t has nothing to move (their weights are zero)
__device__ __forceinline__ bool tile_frozen(const TileSkip &sk, int32_t tile, int t) {
    const uint2 r = sk.tgr[tile];
    for (uint32_t g = r.x; g <= r.y; ++g)
        if (sk.gs[g].stop_after >= t) return false;
    return true;
}

// Scatter step (push): every edge i -> j of a row with w_i != 0 adds w_i to h_j
// with a hardware FP atomic.  Merge-path tiles give every tile the same number
// of rows + edges, so a hub row is spread over many tiles and a run of short
// rows over few.  The tile's target ids are staged in LDS with coalesced
// loads; tiles whose rows are all inactive skip the edge stream.  A capped grid
// loops over the tiles, so a sweep that gathers instead costs one cheap launch.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_push(int t, const Ctl *ctl, int check_mode, const uint32_t *rp,
                                                 int32_t R, const int32_t *col, const uint2 *plan, uint32_t items,
                                                 int32_t ntiles, const T *w, T *h, TileSkip skip) {
    constexpr int IPB = K * kBlock;
    if (t >= 0 && (t > ctl->stop_after || (check_mode && ctl->use_pull))) return;
    __shared__ uint32_t s_end[IPB + 1];
    __shared__ int32_t s_col[IPB];
    __shared__ T s_w[IPB + 1];
    const uint32_t rp0 = rp[0];
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        if (skip.tgr && tile_frozen(skip, tile, t)) continue;  // uniform over the workgroup
        const uint2 a = plan[tile], b = plan[tile + 1];
        const int32_t i0 = (int32_t)a.x;
        const int32_t i1 = min((int32_t)b.x, R - 1);
        const uint32_t e0 = a.y, e1 = b.y;
        const int32_t nr = i1 - i0 + 1;
        int any = 0;
        {
            uint32_t rv[K + 1];
            T wv[K + 1];
#pragma unroll
            for (int j = 0; j <= K; ++j) {
                const int32_t kk = min((int32_t)threadIdx.x + j * kBlock, nr - 1);
                rv[j] = ld_stream(rp + i0 + 1 + kk);
                wv[j] = w[i0 + kk];
            }
#pragma unroll
            for (int j = 0; j <= K; ++j) {
                const int32_t kk = threadIdx.x + j * kBlock;
                if (kk < nr) {
                    s_end[kk] = rv[j] - rp0 + (uint32_t)(i0 + kk);
                    s_w[kk] = wv[j];
                    any |= (wv[j] != (T)0);
                }
            }
        }
        any = __syncthreads_or(any);
        if (!any) continue;  // uniform: every thread saw the same OR
        const int32_t ne = (int32_t)(e1 - e0);
        if (ne > 0) {
            int32_t cv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) cv[j] = ld_stream(col + e0 + min((int32_t)threadIdx.x + j * kBlock, ne - 1));
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int32_t e = threadIdx.x + j * kBlock;
                if (e < ne) s_col[e] = cv[j];
            }
        }
        __syncthreads();
        uint32_t d = min((uint32_t)(tile * IPB + threadIdx.x * K), items);
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
            T wr = k < nr ? s_w[k] : (T)0;
            for (; d < dend; ++d) {
                if (d == s_end[k]) {
                    ++k;
                    wr = k < nr ? s_w[k] : (T)0;
                } else {
                    if (wr != (T)0) atomicAdd(h + s_col[et - e0], wr);
                    ++et;
                }
            }
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// Gather step (pull): out_j += sum over in-edges u -> j of w_u, without global
// atomics except for the first and last row of a tile.  Same merge-path tiling
// as the push; all w_u of a tile's in-edges are first gathered into LDS in one
// batched pass, then each thread walks its rows + edges from LDS, with sums
// carried in FP64.  Every row's sum meets in an LDS accumulator (a plain store
// for a row one thread holds whole, a hardware LDS add for pieces of rows
// shared by threads), and the tile writes its rows out together at the end, so
// a hub row costs one global atomic per tile instead of one per thread.  With rid,
// the plan's rows are only those with an edge in it and rid names their targets.
template <typename WT, typename OT, int K>
__global__ __launch_bounds__(kBlock) void k_pull(int t, const Ctl *ctl, int check_mode, const uint32_t *rp,
                                                 int32_t R, const int32_t *src, const uint2 *plan, uint32_t items,
                                                 int32_t ntiles, const WT *w, OT *out, const int32_t *rid,
                                                 TileSkip skip) {
    constexpr int IPB = K * kBlock;
    static_assert(IPB < 65536, "row ends are kept as 16-bit offsets within the tile");
    // pieces of rows shared by threads meet in FP64, or in FP32 when the output is FP32
    // (the sum is rounded to FP32 when it is added to the output anyway); smaller LDS
    // footprints let more workgroups share a CU
    using AccT = typename std::conditional<sizeof(OT) == 4, float, double>::type;
    if (t >= 0 && (t > ctl->stop_after || (check_mode && !ctl->use_pull))) return;
    // exactly 2 IPB + 4 IPB + 4 IPB bytes (FP32), so that 4 (IPB = 4096) or 8 (2048)
    // workgroups fill the 160 KB of LDS of a CU
    __shared__ uint16_t s_end[IPB];  // row ends in tile items, clamped to IPB
    __shared__ WT s_val[IPB];
    __shared__ AccT s_acc[IPB];
    const uint32_t rp0 = rp[0];
    for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        if (skip.tgr && tile_frozen(skip, tile, t)) continue;  // uniform over the workgroup
        const uint32_t base = (uint32_t)tile * IPB;  // first item of the tile
        const uint2 a = plan[tile], b = plan[tile + 1];
        const int32_t i0 = (int32_t)a.x;
        const int32_t i1 = min((int32_t)b.x, R - 1);
        const uint32_t e0 = a.y, e1 = b.y;
        // A tile of IPB items touches IPB + 1 rows only when all its items end rows
        // i0 .. i0 + IPB - 1 (it holds no edge): row i0 + IPB then has no item here and
        // is left out, so at most IPB rows are kept.
        const int32_t nr = min(i1 - i0 + 1, IPB);
        const uint32_t first = rp[i0];  // first edge of row i0
        const int32_t ne = (int32_t)(e1 - e0);
        // Every load of the tile issues before the first LDS store, indices clamped so
        // that the loads are unconditional and back to back: K row ends (nr <= IPB rows),
        // K coalesced source ids, then K independent weights in flight per thread.
        uint32_t rv[K];
        int32_t sidx[K];
        WT v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) rv[j] = ld_stream(rp + i0 + 1 + min((int32_t)threadIdx.x + j * kBlock, nr - 1));
        if (ne > 0) {  // uniform over the workgroup
#pragma unroll
            for (int j = 0; j < K; ++j) sidx[j] = ld_stream(src + e0 + min((int32_t)threadIdx.x + j * kBlock, ne - 1));
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = w[sidx[j]];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int32_t kk = threadIdx.x + j * kBlock;
            if (kk < nr) {
                // the row of the tile's first item ends at or after it
                s_end[kk] = (uint16_t)min(rv[j] - rp0 + (uint32_t)(i0 + kk) - base, (uint32_t)IPB);
                s_acc[kk] = (AccT)0;
            }
        }
        if (ne > 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int32_t e = threadIdx.x + j * kBlock;
                if (e < ne) s_val[e] = v[j];
            }
        }
        __syncthreads();
        const uint32_t d0 = min(base + threadIdx.x * (uint32_t)K, items);
        const uint32_t dend = min(d0 + (uint32_t)K, items);
        if (d0 < dend) {
            // items of this thread, as offsets within the tile (< IPB)
            uint32_t d = d0 - base;
            const uint32_t dr_end = dend - base;
            int32_t lo = 0, hi = nr;
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (s_end[mid] < d) lo = mid + 1;
                else hi = mid;
            }
            int32_t k = lo;
            uint32_t et = rp0 + d0 - (uint32_t)(i0 + k);
            // first edge of row i0 + k (row k - 1 ends inside the tile)
            uint32_t row_first = k == 0 ? first : (uint32_t)s_end[k - 1] + base + rp0 + 1u - (uint32_t)(i0 + k);
            bool owned = et == row_first;
            bool touched = false;
            double acc = 0.0;
            for (; d < dr_end; ++d) {
                if (d == s_end[k]) {
                    if (touched) {
                        // a row this thread holds whole has no other writer in the tile
                        if (owned) s_acc[k] = (AccT)acc;
                        else atomicAdd(s_acc + k, (AccT)acc);
                    }
                    acc = 0.0;
                    touched = false;
                    owned = true;
                    ++k;
                } else {
                    acc += (double)s_val[et - e0];
                    touched = true;
                    ++et;
                }
            }
            if (touched) atomicAdd(s_acc + k, (AccT)acc);
        }
        __syncthreads();
        // every row's sum goes out here, one coalesced read-modify-write per row (no
        // dependent global loads inside the walk above); rows strictly inside the
        // tile belong to this workgroup alone
        for (int32_t k = threadIdx.x; k < nr; k += kBlock) {
            double v = (double)s_acc[k];
            if (v == 0.0) continue;
            OT *o = out + (rid ? rid[i0 + k] : i0 + k);  // a group plan's rows map to target ids
            if (k == 0 || k == nr - 1) atomicAdd(o, (OT)v);
            else *o = (OT)((double)*o + v);
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// IFP2 phase 2 inputs: w2_u = c z_u / deg(u) for non-dangling u, and the
// initial mass of every dangling vertex.
template <typename T>
__global__ void k_phase2_prep(InitArgs a, const T *h, const double *pibar, const int32_t *deg, double c,
                              int literal, double *w2, double *xD) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        if (i < a.nN) {
            double z = pibar[i] + (literal ? 0.0 : (double)h[i]);
            w2[i] = c * z / (double)deg[i];
        } else {
            xD[i - a.nN] = h0_of<T>(a, i);
        }
    }
}

// a finished level of peeled vertices passes its values on to the levels below
__global__ void k_peel_w2(int32_t lo, int32_t hi, int32_t nN, const double *xD, const int32_t *deg, double c,
                          double *w2) {
    for (int64_t v = lo + blockIdx.x * (int64_t)kBlock + threadIdx.x; v < hi; v += (int64_t)gridDim.x * kBlock)
        w2[v] = c * xD[v - nN] / (double)deg[v];
}

template <typename T>
__device__ __forceinline__ double x_ifp(const InitArgs &a, const T *h, const double *pibar, const double *xD,
                                        int ifp2, int literal, int64_t i) {
    if (i < a.nN) return pibar[i] + (literal ? 0.0 : (double)h[i]);
    return ifp2 ? xD[i - a.nN] : (double)h[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_final_sum(InitArgs a, const T *h, const double *pibar,
                                                      const double *xD, int ifp2, int literal, const float *g,
                                                      double *part) {
    double s = 0.0, sn = 0.0, sa = 0.0, sr = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const double x = x_ifp(a, h, pibar, xD, ifp2, literal, i);
        s += x;
        sa += fabs(x);
        if (i < a.nN) {
            const double r = fabs((double)h[i]);
            sr += r;
            sn += g ? r * (double)g[i] : r;
        }
    }
    __shared__ double sd[4 * (kBlock / W)];
    double v[4] = {s, sn, sa, sr};
    block_sum_n(v, sd);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) part[q * gridDim.x + blockIdx.x] = v[q];
    }
}

// fin_sum = part[0..nb), fin_sn = part[nb..2nb) (weighted residual), fin_abs =
// part[2nb..3nb), fin_res = part[3nb..4nb) (plain residual)
__global__ __launch_bounds__(kBlock) void k_final_decide(Ctl *ctl, int nb, const double *part) {
    __shared__ double sd[4 * (kBlock / W)];
    double v[4];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x == 0) {
        ctl->fin_sum = v[0];
        ctl->fin_sn = v[1];
        ctl->fin_abs = v[2];
        ctl->fin_res = v[3];
    }
}

template <typename T>
__global__ void k_final_write(const Ctl *ctl, InitArgs a, const T *h, const double *pibar, const double *xD,
                              int ifp2, int literal, double *out) {
    const double inv = 1.0 / ctl->fin_sum;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock)
        out[a.perm[i]] = x_ifp(a, h, pibar, xD, ifp2, literal, i) * inv;
}

// ------------------------------------------------------------------------
// power method
// ------------------------------------------------------------------------
__device__ __forceinline__ double p_of(const InitArgs &a, int64_t i) {
    if (a.source >= 0) return a.perm[i] == a.source ? 1.0 : 0.0;
    if (a.uniform) return 1.0 / (double)a.n;
    return a.p[a.perm[i]] * a.pscale;
}

__global__ void k_power_init(InitArgs a, double *x, double *acc) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        x[i] = p_of(a, i);
        acc[i] = 0.0;
    }
}

// Iterate t: x_t = acc + b_{t-1} p (t > 0), ||x_t - x_{t-1}||_1, y = c x_t / deg on
// non-dangling vertices, the dangling mass and total mass for b_t; acc cleared
// for the gather that follows.
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_power_prescale(int t, const Ctl *ctl, InitArgs a, double *x, double *acc,
                                                           WT *y, const int32_t *deg, double c, double *part) {
    if (t > ctl->stop_after) return;
    const double b = ctl->pw_b;
    double diff = 0.0, dsum = 0.0, xsum = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        double xv = x[i];
        if (t > 0) {
            double xn = acc[i] + b * p_of(a, i);
            diff += fabs(xn - xv);
            x[i] = xn;
            xv = xn;
        }
        acc[i] = 0.0;
        xsum += xv;
        if (i < a.nN) y[i] = (WT)(c * xv / (double)deg[i]);
        else dsum += xv;
    }
    __shared__ double sd[kBlock / W];
    diff = block_sum(diff, sd);
    dsum = block_sum(dsum, sd);
    xsum = block_sum(xsum, sd);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = diff;
        part[gridDim.x + blockIdx.x] = dsum;
        part[2 * gridDim.x + blockIdx.x] = xsum;
    }
}

// jump weight b_t = c d^T x_t + (1 - c) e^T x_t for the next iterate; stop when
// c / (1 - c) ||x_t - x_{t-1}||_1 <= tol (x_t is then the answer: skip the gather)
__global__ __launch_bounds__(kBlock) void k_decide_power(int t, Ctl *ctl, int nb, const double *part, double c,
                                                         double tol) {
    if (t > ctl->stop_after) return;
    __shared__ double sd[3 * (kBlock / W)];
    double v[3];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x != 0) return;
    const double df = v[0], ds = v[1], xs = v[2];
    ctl->pw_b = c * ds + (1.0 - c) * xs;
    if (t > 0) {
        ctl->pw_diff = df;
        ctl->sweeps = t;
        ctl->last_bound = c / (1.0 - c) * df;
        if (ctl->last_bound <= tol) ctl->stop_after = t - 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_final_x_sum(int64_t n, const double *x, double *part) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) s += x[i];
    __shared__ double sd[kBlock / W];
    s = block_sum(s, sd);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        part[gridDim.x + blockIdx.x] = 0.0;
        part[2 * gridDim.x + blockIdx.x] = s;  // the iterates are non-negative
        part[3 * gridDim.x + blockIdx.x] = 0.0;
    }
}

__global__ void k_final_x_write(const Ctl *ctl, InitArgs a, const double *x, double *out) {
    const double inv = 1.0 / ctl->fin_sum;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock)
        out[a.perm[i]] = x[i] * inv;
}

// ------------------------------------------------------------------------
// a-posteriori check of a written result (PR_VERIFY): for the normalised output
// pi, one application of the power-method matrix P'' of Eq. 1 gives the residual
// r = P'' pi - pi; since P'' contracts differences of equal sum by c in L1,
// ||pi - pi_exact||_1 <= ||r||_1 / (1 - c) + |sum(pi) - 1|, whatever arithmetic
// produced pi.  A second bound weighs each row instead: for any beta > 0,
// u = pi / beta solves (I - cP) u = p - r_beta / beta with r_beta = beta p -
// (I - cP) pi, so u differs from y = (I - cP)^{-1} p (Eq. 4, dangling vertices
// absorbing) by (I - cP)^{-1} r_beta / beta, whose L1 norm is at most
// sum_j f_j |r_beta,j| / beta with f_j the mass that a unit at j adds to y: 1 at a
// dangling j, and 1 + c delta_j + g_j at a non-dangling one (the stop rule's
// weights, upper bounds).  Normalising, pi_exact = y / |y| and |u| = sum(pi) / beta
// give ||pi - pi_exact||_1 <= 2 sum_j f_j |r_beta,j| / sum(pi) + |sum(pi) - 1|.  Two
// betas are tried: b = c d^T pi + (1 - c) sum(pi) (then r_beta = r), and the ratio
// pi_j / p_j over the vertices without in-edges, where the IFP output is exact
// (their value is the initial mass, which fixes the scale of the unnormalised
// vector; then r_beta is the residual mass the push has not yet delivered, and the
// bound equals the stop rule's).  The rounding of the check itself is bounded row by
// row.
// ------------------------------------------------------------------------
// x = the output in the internal order, acc = 0; partials of sum pi_j and sum p_j over
// the vertices without in-edges
__global__ __launch_bounds__(kBlock) void k_verify_load(InitArgs a, const uint32_t *in_ptr, const double *out,
                                                        double *x, double *acc, double *part) {
    double xs = 0.0, ps = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const double v = out[a.perm[i]];
        x[i] = v;
        acc[i] = 0.0;
        if (in_ptr[i + 1] == in_ptr[i]) {
            xs += v;
            ps += p_of(a, i);
        }
    }
    __shared__ double sd[kBlock / W];
    xs = block_sum(xs, sd);
    ps = block_sum(ps, sd);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = xs;
        part[gridDim.x + blockIdx.x] = ps;
    }
}

// the second beta of the weighted bound (0: none, no vertex without in-edges carries p)
__global__ __launch_bounds__(kBlock) void k_verify_beta(Ctl *ctl, int nb, const double *part) {
    __shared__ double sd[2 * (kBlock / W)];
    double v[2];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x != 0) return;
    ctl->ver_beta = v[1] > 0.0 ? v[0] / v[1] : 0.0;
}

// per row j: r_j = |acc_j + b p_j - x_j| with acc_j = sum over in-edges of c x_u / deg(u);
// err_j bounds the FP64 rounding of computing it: the k_j-term sum of acc_j (any order:
// k_j - 1 additions), the quotients c x_u / deg(u) (2 each), b (depth_b additions of
// its reduction) and the final add, subtract and absolute value (with the larger of the
// two betas, which covers the second residual too).  With weights g (of the first nN
// rows), rf and rf2 accumulate f_j r_j for both betas; f_j is widened by 1e-12
// relative over the rounding of forming it.
__global__ __launch_bounds__(kBlock) void k_verify_residual(const Ctl *ctl, InitArgs a, const uint32_t *in_ptr,
                                                            const double *x, const double *acc, double depth_b,
                                                            double c, const float *g, int32_t nN, const int32_t *deg,
                                                            const uint32_t *rp_nn, double *part) {
    const double b = ctl->pw_b;
    const double b2 = ctl->ver_beta;
    const double bm = fmax(b, b2);
    double r = 0.0, err = 0.0, xs = 0.0, rf = 0.0, rf2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kBlock) {
        const double k = (double)(in_ptr[i + 1] - in_ptr[i]);
        const double pv = p_of(a, i);
        const double ri = fabs(acc[i] + b * pv - x[i]);
        r += ri;
        err += (k + 4.0 + depth_b) * (acc[i] + bm * pv + x[i]);
        xs += x[i];
        if (g) {
            double f = 1.0;
            if (i < nN) {
                const double dg = (double)deg[i];
                const double delta = 1.0 - (double)(rp_nn[i + 1] - rp_nn[i]) / dg;
                f = (1.0 + c * delta + (double)g[i]) * (1.0 + 1e-12);
            }
            rf += f * ri;
            rf2 += f * fabs(acc[i] + b2 * pv - x[i]);
        }
    }
    __shared__ double sd[kBlock / W];
    r = block_sum(r, sd);
    err = block_sum(err, sd);
    xs = block_sum(xs, sd);
    rf = block_sum(rf, sd);
    rf2 = block_sum(rf2, sd);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = r;
        part[gridDim.x + blockIdx.x] = err;
        part[2 * gridDim.x + blockIdx.x] = xs;
        part[3 * gridDim.x + blockIdx.x] = rf;
        part[4 * gridDim.x + blockIdx.x] = rf2;
    }
}

__global__ __launch_bounds__(kBlock) void k_verify_decide(Ctl *ctl, int nb, const double *part) {
    __shared__ double sd[5 * (kBlock / W)];
    double v[5];
    reduce_partials_n(part, nb, v, sd);
    if (threadIdx.x != 0) return;
    ctl->ver_r = v[0];
    ctl->ver_err = v[1];
    ctl->ver_sum = v[2];
    ctl->ver_rf = v[3];
    ctl->ver_rf2 = ctl->ver_beta > 0.0 ? v[4] : INFINITY;
}

// ------------------------------------------------------------------------
// error weights of the stop rule (folded IFP2).  A unit of residual left at a
// non-dangling i would still be pushed: c / deg(i) to each non-dangling out-neighbour
// j, whose arrival then counts itself, the share c delta_j it sends to dangling
// vertices (delta_j: the share of j's out-edges that lead there), and its own pushes
// on.  With f_j the mass a unit arriving at j adds in total,
//   f_j = 1 + c delta_j + (c / deg(j)) sum_{k in out_N(j)} f_k,
// and g_i = (c / deg(i)) sum_{j in out_N(i)} f_j is the error a unit at i leaves.
// f = 1 / (1 - c) satisfies f >= T(f), so the iterates from it decrease to the
// fixed point and each is an upper bound; the stored weights are rounded up with a
// relative margin of 1e-6 over the FP64 rounding of the iterations.
// ------------------------------------------------------------------------
__global__ void k_amp_init(int32_t nN, double c, double *f, double *acc) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nN; i += (int64_t)gridDim.x * kBlock) {
        f[i] = 1.0 / (1.0 - c);
        acc[i] = 0.0;
    }
}

// f_i = 1 + c delta_i + c acc_i / deg(i), acc_i = sum of f over i's N out-neighbours
__global__ void k_amp_step(int32_t nN, double c, const int32_t *deg, const uint32_t *rp_nn, double *f, double *acc) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nN; i += (int64_t)gridDim.x * kBlock) {
        const double dg = (double)deg[i];
        const double delta = 1.0 - (double)(rp_nn[i + 1] - rp_nn[i]) / dg;
        f[i] = 1.0 + c * delta + c * acc[i] / dg;
        acc[i] = 0.0;
    }
}

// g_i = c acc_i / deg(i) (acc = sum of f), rounded up
__global__ void k_amp_g(int32_t nN, double c, const int32_t *deg, double *acc, float *g) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nN; i += (int64_t)gridDim.x * kBlock) {
        g[i] = __double2float_ru(c * acc[i] / (double)deg[i] * (1.0 + 1e-6));
        acc[i] = 0.0;
    }
}

// q_i = acc_i / deg(i) (acc = sum of g), rounded up
__global__ void k_amp_q(int32_t nN, const int32_t *deg, const double *acc, float *q) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < nN; i += (int64_t)gridDim.x * kBlock)
        q[i] = __double2float_ru(acc[i] / (double)deg[i] * (1.0 + 1e-6));
}

// see launch_amp_qle; one wave per vertex, its out-list split over the lanes with eight
// edges per lane in flight (a hub's list of 10^5 edges would take one thread milliseconds);
// built once per graph, factor and grouping; unit weights when g is null
__global__ __launch_bounds__(kBlock) void k_amp_qle(int32_t nN, const uint32_t *rp_nn, const int32_t *col_nn,
                                                    const int32_t *deg, const float *g, GroupEnds ge, float *qle) {
    constexpr int U = 8;
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / W);
    for (int64_t u = blockIdx.x * (int64_t)(kBlock / W) + threadIdx.x / W; u < nN; u += nwaves) {
        int32_t end = nN;
        for (int q = 0; q < ge.ng; ++q)
            if (u < ge.end[q]) {
                end = ge.end[q];
                break;
            }
        const uint32_t e0 = rp_nn[u], e1 = rp_nn[u + 1];
        double s = 0.0;
        for (uint32_t e = e0 + (uint32_t)lane; e < e1; e += U * W) {
            int32_t j[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t ek = e + (uint32_t)(k * W);
                j[k] = ek < e1 ? col_nn[ek] : end;  // past the row: a target that is not counted
            }
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (j[k] < end) s += g ? (double)g[j[k]] : 1.0;
        }
        s = wave_sum(s);
        if (lane == 0) qle[u] = __double2float_ru(s / (double)deg[u] * (1.0 + 1e-6));
    }
}

// fill kernels (clearing counters and sums without a memset node in the stream)
__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t count, double v) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

// p validation: sum_bad[0] += p_i, sum_bad[1] += 1 for every negative or non-finite entry
__global__ __launch_bounds__(kBlock) void k_validate_p(const double *p, int64_t n, double *sum_bad) {
    double s = 0.0, bad = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v = p[i];
        if (!(v >= 0.0) || !isfinite(v)) bad += 1.0;
        else s += v;
    }
    __shared__ double sd[kBlock / W];
    s = block_sum(s, sd);
    bad = block_sum(bad, sd);
    if (threadIdx.x == 0) {
        atomic_add_f64(&sum_bad[0], s);
        if (bad != 0.0) atomic_add_f64(&sum_bad[1], bad);
    }
}

}  // namespace

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
// every kernel launch of this file is counted (the launches field of a solve's stats)
thread_local int64_t t_kernel_launches = 0;
#define PRK_GGL(...)                        \
    do {                                    \
        ++t_kernel_launches;                \
        hipLaunchKernelGGL(__VA_ARGS__);    \
    } while (0)
#define PRK_LAUNCH(kern, grid, ...)                                          \
    do {                                                                     \
        PRK_GGL(kern, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__);          \
        return hipGetLastError();                                            \
    } while (0)

hipError_t launch_check_cols(const int32_t *col, int64_t m, int64_t n, unsigned int *bad, hipStream_t s) {
    if (m == 0) return hipSuccess;
    PRK_LAUNCH(k_check_cols, grid_for(m, 8, 8192), col, m, n, bad);
}
hipError_t launch_degree_class(const int64_t *rp64, int64_t n, uint32_t *isN, hipStream_t s) {
    PRK_LAUNCH(k_degree_class, grid_for(n, 4, 8192), rp64, n, isN);
}
hipError_t launch_indegree(const int32_t *col, int64_t m, uint32_t *indeg, hipStream_t s) {
    if (m == 0) return hipSuccess;
    PRK_LAUNCH(k_indegree, grid_for(m, 8, 8192), col, m, indeg);
}
size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
    if (n == 0) {
        // out[0] = 0
        return hipMemsetAsync(out, 0, sizeof(uint32_t), s);
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    PRK_GGL(k_scan_partial, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tmp);
    PRK_GGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tmp, nb);
    PRK_GGL(k_scan_final, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, (const uint32_t *)tmp);
    return hipGetLastError();
}
hipError_t launch_relabel(const uint32_t *isN, const uint32_t *rankN, int64_t n, int32_t nN, int32_t *newid,
                          int32_t *perm, hipStream_t s) {
    PRK_LAUNCH(k_relabel, grid_for(n, 4, 8192), isN, rankN, n, nN, newid, perm);
}
hipError_t launch_count_nn(const int64_t *rp64, const int32_t *col, const uint32_t *isN, const int32_t *perm,
                           int32_t nN, uint32_t *cnt_nn, uint32_t *cnt_nd, int32_t *deg, hipStream_t s) {
    if (nN == 0) return hipSuccess;
    PRK_LAUNCH(k_count_nn, grid_for((int64_t)nN * W, 1, 16384), rp64, col, isN, perm, nN, cnt_nn, cnt_nd, deg);
}
hipError_t launch_split_rows(const int64_t *rp64, const int32_t *col, const uint32_t *isN, const int32_t *newid,
                             const int32_t *perm, int32_t nN, const uint32_t *rp_nn, int32_t *col_nn,
                             const uint32_t *rp_nd, int32_t *col_nd, hipStream_t s) {
    if (nN == 0) return hipSuccess;
    PRK_LAUNCH(k_split_rows, grid_for((int64_t)nN * W, 1, 16384), rp64, col, isN, newid, perm, nN, rp_nn, col_nn,
               rp_nd, col_nd);
}
hipError_t launch_permute_u32(const uint32_t *in_old, const int32_t *perm, int64_t n, uint32_t *out_new,
                              hipStream_t s) {
    PRK_LAUNCH(k_permute_u32, grid_for(n, 4, 8192), in_old, perm, n, out_new);
}
hipError_t launch_fill_csc(const uint32_t *rp, const int32_t *col, int32_t R, uint32_t *cursor, int32_t *in_src,
                           hipStream_t s) {
    if (R == 0) return hipSuccess;
    PRK_LAUNCH(k_fill_csc, grid_for((int64_t)R * W, 1, 16384), rp, col, R, cursor, in_src);
}
hipError_t launch_count_zero(const uint32_t *a, int64_t n, unsigned long long *out, hipStream_t s) {
    PRK_LAUNCH(k_count_zero, grid_for(n, 8, 4096), a, n, out);
}
hipError_t launch_depth_init(int32_t nN, const uint32_t *in_ptr, uint32_t *rem, int32_t *depth, int32_t *q,
                             uint32_t *qcount, hipStream_t s) {
    if (nN == 0) return hipSuccess;
    PRK_LAUNCH(k_depth_init, grid_for(nN, 4, 8192), nN, in_ptr, rem, depth, q, qcount);
}
hipError_t launch_depth_step(const int32_t *q, uint32_t qsize, const uint32_t *rp_nn, const int32_t *col_nn,
                             uint32_t *rem, int32_t *depth, int32_t round, int32_t *next, uint32_t *ncount,
                             hipStream_t s) {
    if (qsize == 0) return hipSuccess;
    PRK_LAUNCH(k_depth_step, grid_for((int64_t)qsize * W, 1, 16384), q, qsize, rp_nn, col_nn, rem, depth, round, next,
               ncount);
}
hipError_t launch_live_count(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                             int32_t t0, int32_t slo, int32_t shi, uint32_t *cnt, hipStream_t s, const uint8_t *grp,
                             int32_t q) {
    if (R == 0) return hipSuccess;
    PRK_LAUNCH(k_live_count, grid_for((int64_t)R * W, 1, 16384), R, in_ptr, in_src, depth, t0, slo, shi, grp, q,
               cnt);
}
hipError_t launch_live_fill(int32_t R, const uint32_t *in_ptr, const int32_t *in_src, const int32_t *depth,
                            int32_t t0, int32_t slo, int32_t shi, const uint32_t *out_ptr, int32_t *out_src,
                            hipStream_t s, const uint8_t *grp, int32_t q) {
    if (R == 0) return hipSuccess;
    PRK_LAUNCH(k_live_fill, grid_for((int64_t)R * W, 1, 16384), R, in_ptr, in_src, depth, t0, slo, shi, grp, q,
               out_ptr, out_src);
}
hipError_t launch_row_flags(int32_t R, const uint32_t *cnt, uint32_t *flag, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    PRK_LAUNCH(k_row_flags, grid_for(R, 4, 8192), R, cnt, flag);
}
hipError_t launch_row_fill(int32_t R, const uint32_t *cnt, const uint32_t *pos, const uint32_t *off, int32_t *rid,
                           uint32_t *rp, hipStream_t s) {
    PRK_LAUNCH(k_row_fill, grid_for((int64_t)R + 1, 4, 8192), R, cnt, pos, off, rid, rp);
}
hipError_t launch_plan(MPPlan &p, hipStream_t s) {
    p.blocks = (int32_t)(((int64_t)p.items + p.ipb - 1) / p.ipb);
    PRK_LAUNCH(k_plan, grid_for((int64_t)p.blocks + 1, 1, 4096), p.rp, p.R, p.items, p.ipb, p.blocks, p.plan);
}

template <typename T>
hipError_t launch_init_ifp(const InitArgs &a, T *h, double *pibar, hipStream_t s) {
    PRK_LAUNCH(k_init_ifp<T>, grid_for(a.n, 4, 8192), a, h, pibar);
}

template <typename T>
hipError_t launch_reserve(int t, Ctl *ctl, Trace *tr, int32_t nN, T *h, T *w, double *pibar, const int32_t *deg,
                          const uint32_t *rp_nn, double c, double xi, int ifp2, ErrWeights ew, double kb,
                          int stop_l1, double tol, unsigned long long pull_edges_thr, int force,
                          unsigned long long pull_edges, double *part, hipStream_t s) {
    const int nb = grid_for(nN, 4, kRedBlocks);
    PRK_GGL(k_reserve<T>, dim3(nb), dim3(kBlock), 0, s, t, (const Ctl *)ctl, 0, nN, h, w, pibar, deg,
                       rp_nn, c, (T)xi, ifp2, ew, part);
    PRK_GGL(k_decide_ifp, dim3(1), dim3(kBlock), 0, s, t, ctl, tr, nb, (const double *)part, c, kb, stop_l1,
                       tol, pull_edges_thr, force, pull_edges);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reserve_range(int t, Ctl *ctl, int32_t lo, int32_t hi, T *h, T *w, double *pibar,
                                const int32_t *deg, const uint32_t *rp_nn, double c, double xi, int ifp2, int nbg,
                                ErrWeights ew, double *part, hipStream_t s) {
    PRK_GGL(k_reserve<T>, dim3(nbg), dim3(kBlock), 0, s, t, (const Ctl *)ctl, lo, hi, h, w, pibar, deg,
                       rp_nn, c, (T)xi, ifp2, ew, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_decide_gs(int t, Ctl *ctl, Trace *tr, int32_t nN, const T *h, int ng, const GroupBlocks &gb,
                            const double *part, double *part_s, double c, const float *g, double kb, int stop_l1,
                            double tol, unsigned long long pull_thr, unsigned long long pull_edges, int bookkeep,
                            hipStream_t s) {
    const int nbs = bookkeep ? 0 : grid_for(nN, 8, kRedBlocks);
    if (!bookkeep) PRK_GGL(k_sum_h<T>, dim3(nbs), dim3(kBlock), 0, s, t, (const Ctl *)ctl, nN, h, g, part_s);
    PRK_GGL(k_decide_gs, dim3(1), dim3(kBlock), 0, s, t, ctl, tr, ng, gb, part, nbs,
                       (const double *)part_s, c, kb, stop_l1, tol, pull_thr, pull_edges, bookkeep);
    return hipGetLastError();
}

// a launch that is timed takes its start / stop timestamps itself
template <typename F, typename... Args>
hipError_t launch_timed(F kern, int grid, hipStream_t s, KernelEvents ev, Args... args) {
    if (ev.a || ev.b) {
        ++t_kernel_launches;
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, ev.a, ev.b, 0, args...);
    } else {
        PRK_GGL(kern, dim3(grid), dim3(kBlock), 0, s, args...);
    }
    return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_push_k(int t, const Ctl *ctl, const MPPlan &p, const T *w, T *h, int check_mode, hipStream_t s,
                         TileSkip skip, KernelEvents ev) {
    auto kern = &k_push<T, K>;
    static const int grid = resident_grid(kern);
    return launch_timed(kern, std::min(p.blocks, grid), s, ev, t, ctl, check_mode, p.rp, p.R, p.idx,
                        (const uint2 *)p.plan, p.items, p.blocks, w, h, skip);
}

template <typename T>
hipError_t launch_push(int t, const Ctl *ctl, const MPPlan &p, const T *w, T *h, int check_mode, hipStream_t s,
                       TileSkip skip, KernelEvents ev) {
    if (p.blocks == 0 || p.edges() == 0) return hipSuccess;
    switch (p.ipb / kBlock) {
        case 4: return launch_push_k<T, 4>(t, ctl, p, w, h, check_mode, s, skip, ev);
        case 16: return launch_push_k<T, 16>(t, ctl, p, w, h, check_mode, s, skip, ev);
        default: return launch_push_k<T, 8>(t, ctl, p, w, h, check_mode, s, skip, ev);
    }
}

template <typename WT, typename OT, int K>
hipError_t launch_pull_k(int t, const Ctl *ctl, const MPPlan &p, const WT *w, OT *out, int check_mode,
                         hipStream_t s, TileSkip skip, KernelEvents ev) {
    auto kern = &k_pull<WT, OT, K>;
    static const int grid = resident_grid(kern);
    return launch_timed(kern, std::min(p.blocks, grid), s, ev, t, ctl, check_mode, p.rp, p.R, p.idx,
                        (const uint2 *)p.plan, p.items, p.blocks, w, out, p.rid, skip);
}

template <typename WT, typename OT>
hipError_t launch_pull(int t, const Ctl *ctl, const MPPlan &p, const WT *w, OT *out, int check_mode,
                       hipStream_t s, TileSkip skip, KernelEvents ev) {
    if (p.blocks == 0 || p.edges() == 0) return hipSuccess;
    switch (p.ipb / kBlock) {
        case 4: return launch_pull_k<WT, OT, 4>(t, ctl, p, w, out, check_mode, s, skip, ev);
        case 16: return launch_pull_k<WT, OT, 16>(t, ctl, p, w, out, check_mode, s, skip, ev);
        default: return launch_pull_k<WT, OT, 8>(t, ctl, p, w, out, check_mode, s, skip, ev);
    }
}

template <typename T>
hipError_t launch_phase2_prep(const InitArgs &a, const T *h, const double *pibar, const int32_t *deg, double c,
                              int literal, double *w2, double *xD, hipStream_t s) {
    PRK_LAUNCH(k_phase2_prep<T>, grid_for(a.n, 4, 8192), a, h, pibar, deg, c, literal, w2, xD);
}

hipError_t launch_peel_w2(int32_t lo, int32_t hi, int32_t nN, const double *xD, const int32_t *deg, double c,
                          double *w2, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    PRK_LAUNCH(k_peel_w2, grid_for((int64_t)hi - lo, 4, 8192), lo, hi, nN, xD, deg, c, w2);
}

template <typename T>
hipError_t launch_final_ifp(Ctl *ctl, const InitArgs &a, const T *h, const double *pibar, const double *xD,
                            int ifp2, int literal, const float *g, double *out, double *part, hipStream_t s) {
    const int nb = grid_for(a.n, 4, kRedBlocks);
    PRK_GGL(k_final_sum<T>, dim3(nb), dim3(kBlock), 0, s, a, h, pibar, xD, ifp2, literal, g, part);
    PRK_GGL(k_final_decide, dim3(1), dim3(kBlock), 0, s, ctl, nb, (const double *)part);
    PRK_GGL(k_final_write<T>, dim3(grid_for(a.n, 4, 8192)), dim3(kBlock), 0, s, (const Ctl *)ctl, a, h,
                       pibar, xD, ifp2, literal, out);
    return hipGetLastError();
}

hipError_t launch_power_init(const InitArgs &a, double *x, double *acc, hipStream_t s) {
    PRK_LAUNCH(k_power_init, grid_for(a.n, 4, 8192), a, x, acc);
}

template <typename WT>
hipError_t launch_power_prescale(int t, Ctl *ctl, const InitArgs &a, double *x, double *acc, WT *y,
                                 const int32_t *deg, double c, double tol, double *part, hipStream_t s) {
    const int nb = grid_for(a.n, 4, kRedBlocks);
    PRK_GGL(k_power_prescale<WT>, dim3(nb), dim3(kBlock), 0, s, t, (const Ctl *)ctl, a, x, acc, y, deg, c,
                       part);
    PRK_GGL(k_decide_power, dim3(1), dim3(kBlock), 0, s, t, ctl, nb, (const double *)part, c, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_compact(Ctl *ctl, int slot, int32_t nN, const T *h, double xi, int32_t *f, const int32_t *deg,
                          const uint32_t *rp_nn, int ifp2, const float *g, double *part, hipStream_t s) {
    if (nN <= 0) return hipSuccess;
    const int nb = grid_for(nN, 4, kRedBlocks);
    PRK_GGL(k_compact<T>, dim3(nb), dim3(kBlock), 0, s, ctl, slot, nN, h, (T)xi, f, deg, rp_nn, ifp2, g, part);
    PRK_GGL(k_list_start, dim3(1), dim3(kBlock), 0, s, ctl, nb, (const double *)part);
    return hipGetLastError();
}

constexpr int kListBlocks = 512;  // workgroups of the list reserve (its partials feed the decision)

template <typename T>
hipError_t launch_reserve_list(int t, Ctl *ctl, Trace *tr, const ListBufs<T> &lb, T *h, double *pibar,
                               const int32_t *deg, const uint32_t *rp_nn, double c, double xi, int ifp2,
                               ErrWeights ew, double kb, int stop_l1, double tol, double *part, hipStream_t s) {
    static_assert(kListBlocks <= kRedBlocks, "partials");
    PRK_GGL(k_reserve_list<T>, dim3(kListBlocks), dim3(kBlock), 0, s, t, ctl, lb, h, pibar, deg, rp_nn, c, (T)xi,
            ifp2, ew, part);
    PRK_GGL(k_decide_list, dim3(1), dim3(kBlock), 0, s, t, ctl, tr, kListBlocks, (const double *)part, c, kb,
            stop_l1, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_push_list(int t, Ctl *ctl, const ListBufs<T> &lb, T *h, const int32_t *deg, const uint32_t *rp_nn,
                            const int32_t *col_nn, const uint32_t *rp_nd, const int32_t *col_nd, double xi, int ifp2,
                            hipStream_t s) {
    static const int grid = resident_grid(k_push_list<T>);
    PRK_LAUNCH(k_push_list<T>, grid, t, ctl, lb, h, deg, rp_nn, col_nn, rp_nd, col_nd, (T)xi, ifp2);
}

hipError_t launch_amp_weights(int32_t nN, const MPPlan &push_nn, const int32_t *deg, const uint32_t *rp_nn,
                              double c, int iters, double *f, double *acc, float *g, float *q, hipStream_t s) {
    if (nN <= 0) return hipSuccess;
    const int grid = grid_for(nN, 4, 8192);
    PRK_GGL(k_amp_init, dim3(grid), dim3(kBlock), 0, s, nN, c, f, acc);
    for (int k = 0; k < iters; ++k) {
        hipError_t e = launch_pull<double, double>(-1, nullptr, push_nn, f, acc, 0, s);
        if (e != hipSuccess) return e;
        PRK_GGL(k_amp_step, dim3(grid), dim3(kBlock), 0, s, nN, c, deg, rp_nn, f, acc);
    }
    hipError_t e = launch_pull<double, double>(-1, nullptr, push_nn, f, acc, 0, s);
    if (e != hipSuccess) return e;
    PRK_GGL(k_amp_g, dim3(grid), dim3(kBlock), 0, s, nN, c, deg, acc, g);
    e = launch_pull<float, double>(-1, nullptr, push_nn, g, acc, 0, s);
    if (e != hipSuccess) return e;
    PRK_GGL(k_amp_q, dim3(grid), dim3(kBlock), 0, s, nN, deg, (const double *)acc, q);
    return hipGetLastError();
}

hipError_t launch_amp_qle(int32_t nN, const uint32_t *rp_nn, const int32_t *col_nn, const int32_t *deg,
                          const float *g, const GroupEnds &ge, float *qle, hipStream_t s) {
    if (nN <= 0) return hipSuccess;
    PRK_LAUNCH(k_amp_qle, grid_for((int64_t)nN * W, 1, 16384), nN, rp_nn, col_nn, deg, g, ge, qle);
}

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    PRK_LAUNCH(k_fill_u32, grid_for(count, 4, 1024), p, count, 0u);
}

hipError_t launch_zero_f64(double *p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    PRK_LAUNCH(k_fill_f64, grid_for(count, 4, 1024), p, count, 0.0);
}

hipError_t launch_verify(Ctl *vctl, const InitArgs &a, const double *out, double *x, double *acc, double *y,
                         const int32_t *deg, const MPPlan &pull_all, const uint32_t *in_ptr, double c, const float *g,
                         int32_t nN, const uint32_t *rp_nn, double *part, double *depth, hipStream_t s) {
    const int nb = grid_for(a.n, 4, kRedBlocks);
    // depth of a reduction over n entries as the sums below run it: a thread's strided
    // run, the workgroup tree, and the partials summed by one thread per lane
    *depth = (double)((a.n + (int64_t)nb * kBlock - 1) / ((int64_t)nb * kBlock)) + 8.0 + (double)nb;
    PRK_GGL(k_verify_load, dim3(nb), dim3(kBlock), 0, s, a, in_ptr, out, x, acc, part);
    PRK_GGL(k_verify_beta, dim3(1), dim3(kBlock), 0, s, vctl, nb, (const double *)part);
    PRK_GGL(k_power_prescale<double>, dim3(nb), dim3(kBlock), 0, s, 0, (const Ctl *)vctl, a, x, acc, y, deg, c,
            part);
    PRK_GGL(k_decide_power, dim3(1), dim3(kBlock), 0, s, 0, vctl, nb, (const double *)part, c, 0.0);
    hipError_t e = launch_pull<double, double>(0, vctl, pull_all, y, acc, 0, s);
    if (e != hipSuccess) return e;
    PRK_GGL(k_verify_residual, dim3(nb), dim3(kBlock), 0, s, (const Ctl *)vctl, a, in_ptr, (const double *)x,
            (const double *)acc, *depth, c, g, nN, deg, rp_nn, part);
    PRK_GGL(k_verify_decide, dim3(1), dim3(kBlock), 0, s, vctl, nb, (const double *)part);
    return hipGetLastError();
}

hipError_t launch_final_x(Ctl *ctl, const InitArgs &a, const double *x, double *out, double *part, hipStream_t s) {
    const int nb = grid_for(a.n, 4, kRedBlocks);
    PRK_GGL(k_final_x_sum, dim3(nb), dim3(kBlock), 0, s, a.n, x, part);
    PRK_GGL(k_final_decide, dim3(1), dim3(kBlock), 0, s, ctl, nb, (const double *)part);
    PRK_GGL(k_final_x_write, dim3(grid_for(a.n, 4, 8192)), dim3(kBlock), 0, s, (const Ctl *)ctl, a, x,
                       out);
    return hipGetLastError();
}

// out = e_src: the PageRank of a single-source query whose source has no out-edges
__global__ __launch_bounds__(kBlock) void k_unit_vector(double *out, int64_t n, int64_t src) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = i == src ? 1.0 : 0.0;
}

hipError_t launch_unit_vector(double *out, int64_t n, int64_t src, hipStream_t s) {
    PRK_LAUNCH(k_unit_vector, grid_for(n, 4, 4096), out, n, src);
}

hipError_t launch_validate_p(const double *p, int64_t n, double *sum_bad, hipStream_t s) {
    PRK_LAUNCH(k_validate_p, grid_for(n, 4, 2048), p, n, sum_bad);
}

// explicit instantiations
template hipError_t launch_compact<float>(Ctl *, int, int32_t, const float *, double, int32_t *, const int32_t *,
                                          const uint32_t *, int, const float *, double *, hipStream_t);
template hipError_t launch_compact<double>(Ctl *, int, int32_t, const double *, double, int32_t *, const int32_t *,
                                           const uint32_t *, int, const float *, double *, hipStream_t);
template hipError_t launch_reserve_list<float>(int, Ctl *, Trace *, const ListBufs<float> &, float *, double *,
                                               const int32_t *, const uint32_t *, double, double, int, ErrWeights,
                                               double, int, double, double *, hipStream_t);
template hipError_t launch_reserve_list<double>(int, Ctl *, Trace *, const ListBufs<double> &, double *, double *,
                                                const int32_t *, const uint32_t *, double, double, int, ErrWeights,
                                                double, int, double, double *, hipStream_t);
template hipError_t launch_push_list<float>(int, Ctl *, const ListBufs<float> &, float *, const int32_t *,
                                            const uint32_t *, const int32_t *, const uint32_t *, const int32_t *,
                                            double, int, hipStream_t);
template hipError_t launch_push_list<double>(int, Ctl *, const ListBufs<double> &, double *, const int32_t *,
                                             const uint32_t *, const int32_t *, const uint32_t *, const int32_t *,
                                             double, int, hipStream_t);
template hipError_t launch_init_ifp<float>(const InitArgs &, float *, double *, hipStream_t);
template hipError_t launch_init_ifp<double>(const InitArgs &, double *, double *, hipStream_t);
template hipError_t launch_reserve<float>(int, Ctl *, Trace *, int32_t, float *, float *, double *, const int32_t *,
                                          const uint32_t *, double, double, int, ErrWeights, double, int, double,
                                          unsigned long long, int, unsigned long long, double *, hipStream_t);
template hipError_t launch_reserve<double>(int, Ctl *, Trace *, int32_t, double *, double *, double *,
                                           const int32_t *, const uint32_t *, double, double, int, ErrWeights, double,
                                           int, double, unsigned long long, int, unsigned long long, double *,
                                           hipStream_t);
template hipError_t launch_reserve_range<float>(int, Ctl *, int32_t, int32_t, float *, float *, double *,
                                                const int32_t *, const uint32_t *, double, double, int, int,
                                                ErrWeights, double *, hipStream_t);
template hipError_t launch_reserve_range<double>(int, Ctl *, int32_t, int32_t, double *, double *, double *,
                                                 const int32_t *, const uint32_t *, double, double, int, int,
                                                 ErrWeights, double *, hipStream_t);
template hipError_t launch_decide_gs<float>(int, Ctl *, Trace *, int32_t, const float *, int, const GroupBlocks &,
                                            const double *, double *, double, const float *, double, int, double,
                                            unsigned long long, unsigned long long, int, hipStream_t);
template hipError_t launch_decide_gs<double>(int, Ctl *, Trace *, int32_t, const double *, int, const GroupBlocks &,
                                             const double *, double *, double, const float *, double, int, double,
                                             unsigned long long, unsigned long long, int, hipStream_t);

template hipError_t launch_push<float>(int, const Ctl *, const MPPlan &, const float *, float *, int, hipStream_t,
                                       TileSkip, KernelEvents);
template hipError_t launch_push<double>(int, const Ctl *, const MPPlan &, const double *, double *, int,
                                        hipStream_t, TileSkip, KernelEvents);
template hipError_t launch_pull<float, float>(int, const Ctl *, const MPPlan &, const float *, float *, int,
                                              hipStream_t, TileSkip, KernelEvents);
template hipError_t launch_pull<double, double>(int, const Ctl *, const MPPlan &, const double *, double *, int,
                                                hipStream_t, TileSkip, KernelEvents);
template hipError_t launch_pull<float, double>(int, const Ctl *, const MPPlan &, const float *, double *, int,
                                               hipStream_t, TileSkip, KernelEvents);
template hipError_t launch_phase2_prep<float>(const InitArgs &, const float *, const double *, const int32_t *,
                                              double, int, double *, double *, hipStream_t);
template hipError_t launch_phase2_prep<double>(const InitArgs &, const double *, const double *, const int32_t *,
                                               double, int, double *, double *, hipStream_t);
template hipError_t launch_final_ifp<float>(Ctl *, const InitArgs &, const float *, const double *, const double *,
                                            int, int, const float *, double *, double *, hipStream_t);
template hipError_t launch_final_ifp<double>(Ctl *, const InitArgs &, const double *, const double *,
                                             const double *, int, int, const float *, double *, double *, hipStream_t);
template hipError_t launch_power_prescale<float>(int, Ctl *, const InitArgs &, double *, double *, float *,
                                                 const int32_t *, double, double, double *, hipStream_t);
template hipError_t launch_power_prescale<double>(int, Ctl *, const InitArgs &, double *, double *, double *,
                                                  const int32_t *, double, double, double *, hipStream_t);

}  // namespace prk
