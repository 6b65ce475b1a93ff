// pr_set.hip -- kernels of the multi-graph solve (include/pr_set.h): k
// independent graphs uploaded as one block-diagonal union whose device order
// is [non-dangling vertices of graph 0, of graph 1, ...][dangling vertices of
// graph 0, of graph 1, ...].  The edge sweeps (merge-path push and pull of
// pr_kernels.hip) run over the union unchanged: no edge crosses two graphs.
// What is per graph -- damping factor, threshold, the reductions behind the
// stop rule (section 3 of the paper, applied to each graph on its own), the
// stop itself and the normalisation of Eq. 4 -- is handled here, with the
// graph of a union position found by binary search over segment offsets.
#include <hip/hip_runtime.h>

#include <stddef.h>

#include <climits>

#include "pr_device.h"
#include "pr_internal.h"

namespace prk {
namespace {

// graph of union position i in a segment table off[0..k] (off[k] = end): the
// last g with off[g] <= i, so empty segments are skipped
__device__ __forceinline__ int32_t graph_of(const int32_t *off, int32_t k, int64_t i) {
    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Walks increasing positions of one thread; re-searches only past the end of
// the current graph's segment.
struct GraphCursor {
    const int32_t *off;
    int32_t k;
    int32_t g = -1;
    int64_t end = 0;
    __device__ bool advance(int64_t i) {  // true when the graph changed
        if (i < end) return false;
        g = graph_of(off, k, i);
        end = off[g + 1];
        return true;
    }
};

// Per-workgroup accumulation of per-graph sums over a contiguous range of
// positions into NV consecutive doubles of SetG starting at double index fo:
// LDS slots for the first kLG graphs of the range, global FP64 atomics beyond
// (a range covering more than kLG graphs is made of tiny graphs).
constexpr int kLG = 64;
template <int NV>
struct SegAcc {
    double *s;  // LDS, kLG * NV
    SetG *gs;
    int fo;
    int32_t g_lo;
    __device__ double *field(int32_t g, int j) const { return reinterpret_cast<double *>(gs + g) + fo + j; }
    __device__ void add(int32_t g, const double *v) const {
        const int32_t r = g - g_lo;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            if (v[j] == 0.0) continue;
            if (r >= 0 && r < kLG) atomicAdd(s + r * NV + j, v[j]);
            else atomic_add_f64(field(g, j), v[j]);
        }
    }
    // after a barrier: the LDS slots of graphs g_lo .. g_hi go to device memory
    __device__ void flush(int32_t g_hi) const {
        const int ng = min(g_hi - g_lo + 1, kLG);
        for (int j = threadIdx.x; j < ng * NV; j += kBlock) {
            const double v = s[j];
            if (v != 0.0) atomic_add_f64(field(g_lo + j / NV, j % NV), v);
        }
    }
};

// block-contiguous position range of this workgroup over [0, n), whole waves
__device__ __forceinline__ void block_range(int64_t n, int64_t &lo, int64_t &hi) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t chunk = (per + kBlock - 1) / kBlock * kBlock;
    lo = min(n, (int64_t)blockIdx.x * chunk);
    hi = min(n, lo + chunk);
}

}  // namespace

// first and last graph of the rows of every merge-path tile of a plan over the
// non-dangling rows (same row range as the sweep kernels take for a tile)
__global__ void k_set_tile_graphs(const uint2 *plan, int32_t blocks, int32_t R, const int32_t *offN, int32_t k,
                                  uint2 *out) {
    for (int32_t b = blockIdx.x * kBlock + threadIdx.x; b < blocks; b += gridDim.x * kBlock) {
        const int32_t i0 = min((int32_t)plan[b].x, R - 1);
        const int32_t i1 = min((int32_t)plan[b + 1].x, R - 1);
        out[b] = make_uint2((uint32_t)graph_of(offN, k, i0), (uint32_t)graph_of(offN, k, i1));
    }
}

// h = h0 = n_g p_i = 1 for every vertex (uniform personalisation), pibar = 0
template <typename T>
__global__ void k_set_init(int64_t n, int32_t nN, T *h, double *pibar) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        h[i] = (T)1;
        if (i < nN) pibar[i] = 0.0;
    }
}

// Reserve step of one sweep for every graph still running: a non-dangling i of
// graph g with h_i > xi_g moves its residual into pibar_i and publishes
// w_i = c_g v / deg(i); graphs that stopped publish zeros (their scatter adds
// nothing).  Per-graph sums (inactive residual, mass sent to non-dangling
// vertices, growth of the total mass, pushes, pushed edges) go to acc of SetG.
// The positions [0, len) are cut into per-graph segments by pos_off; position p
// of graph g is vertex p + base[g]: all non-dangling vertices (base NULL), or
// one vertex group of every graph (an ordered sweep).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_reserve(int t, const Ctl *ctl, SetG *gs, const int32_t *pos_off,
                                                        const int32_t *base, int32_t k, int32_t len, T *h, T *w,
                                                        double *pibar, const int32_t *deg, const uint32_t *rp_nn) {
    if (t > ctl->stop_after) return;
    int64_t lo, hi;
    block_range(len, lo, hi);
    if (lo >= hi) return;  // whole workgroup
    {
        // graphs that stopped before sweep t - 1 already publish zero weights
        const int32_t g0 = graph_of(pos_off, k, lo), g1 = graph_of(pos_off, k, hi - 1);
        bool idle = true;
        for (int32_t g = g0; g <= g1 && idle; ++g) idle = gs[g].stop_after < t - 1;
        if (idle) return;  // same answer for every thread of the workgroup
    }
    __shared__ double s_acc[kLG * 5];
    for (int j = threadIdx.x; j < kLG * 5; j += kBlock) s_acc[j] = 0.0;
    __syncthreads();
    SegAcc<5> sa{s_acc, gs, (int)(offsetof(SetG, acc) / sizeof(double)), graph_of(pos_off, k, lo)};
    GraphCursor cur{pos_off, k};
    T xi = (T)0;
    double c = 0.0;
    bool live = false;
    int64_t shift = 0;
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // dense set frontier (the last decision gathered): most vertices are taken, so a
    // vertex's degree, row offsets and pibar are loaded with its residual
    const bool eager = ctl->use_pull != 0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBlock) {
        if (cur.g >= 0 && p >= cur.end) {
            sa.add(cur.g, a);
#pragma unroll
            for (int j = 0; j < 5; ++j) a[j] = 0.0;
        }
        if (cur.advance(p)) {
            const SetG &G = gs[cur.g];
            xi = (T)G.xi;
            c = G.c;
            live = G.stop_after >= t;
            shift = base ? base[cur.g] : 0;
        }
        const int64_t i = p + shift;
        const T hv = h[i];
        int32_t dg = 0;
        uint32_t r0 = 0, r1 = 0;
        double pb = 0.0;
        if (eager) {
            dg = deg[i];
            r0 = rp_nn[i];
            r1 = rp_nn[i + 1];
            pb = pibar[i];
        }
        if (live && hv > xi) {
            if (!eager) {
                dg = deg[i];
                r0 = rp_nn[i];
                r1 = rp_nn[i + 1];
                pb = pibar[i];
            }
            const uint32_t dnn = r1 - r0;
            const double v = (double)hv;
            pibar[i] = pb + v;
            h[i] = (T)0;
            w[i] = (T)(c * v / (double)dg);
            const double fN = (double)dnn / (double)dg;
            a[1] += v * fN;
            a[2] += v * fN;
            a[3] += 1.0;
            a[4] += (double)dnn;
        } else {
            w[i] = (T)0;
            if (live) a[0] += (double)hv;
        }
    }
    if (cur.g >= 0) sa.add(cur.g, a);
    __syncthreads();
    sa.flush(graph_of(pos_off, k, hi - 1));
}

// Residual left on each running graph's non-dangling vertices after an ordered
// sweep, summed directly (mass one group pushes may already have been taken by
// a later group of the same sweep): SetG::sn, cleared again by the decision.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_sum_h(int t, const Ctl *ctl, SetG *gs, const int32_t *offN,
                                                      int32_t k, int32_t nN, const T *h) {
    if (t > ctl->stop_after) return;
    int64_t lo, hi;
    block_range(nN, lo, hi);
    if (lo >= hi) return;
    {
        const int32_t g0 = graph_of(offN, k, lo), g1 = graph_of(offN, k, hi - 1);
        bool idle = true;
        for (int32_t g = g0; g <= g1 && idle; ++g) idle = gs[g].stop_after < t;
        if (idle) return;
    }
    __shared__ double s_acc[kLG];
    for (int j = threadIdx.x; j < kLG; j += kBlock) s_acc[j] = 0.0;
    __syncthreads();
    SegAcc<1> sa{s_acc, gs, (int)(offsetof(SetG, sn) / sizeof(double)), graph_of(offN, k, lo)};
    GraphCursor cur{offN, k};
    bool live = false;
    double a = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        if (cur.g >= 0 && i >= cur.end) {
            sa.add(cur.g, &a);
            a = 0.0;
        }
        if (cur.advance(i)) live = gs[cur.g].stop_after >= t;
        if (live) a += fabs((double)h[i]);
    }
    if (cur.g >= 0) sa.add(cur.g, &a);
    __syncthreads();
    sa.flush(graph_of(offN, k, hi - 1));
}

// Management step of one sweep (one workgroup of 1024): for every running
// graph the certified bound after this sweep's pushes and its stop; then the
// union's push/pull mode: gather when the pushed edges reach half of what a
// gather reads, i.e. of the live edges of the graphs whose scatter this sweep
// still counts (tiles of the others are skipped).  Accumulators are cleared
// for the next sweep.  After an ordered sweep the residual on the non-dangling
// vertices is the directly summed SetG::sn.
constexpr int kDecideThreads = 1024;
__global__ __launch_bounds__(kDecideThreads) void k_set_decide(int t, Ctl *ctl, SetG *gs, int32_t k, int stop_l1,
                                                               double tol, double live_frac, int force,
                                                               int ordered) {
    if (t > ctl->stop_after) return;
    double edges = 0.0, running = 0.0, bmax = 0.0, live = 0.0;
    for (int32_t g = threadIdx.x; g < k; g += kDecideThreads) {
        SetG &S = gs[g];
        if (S.stop_after < t) continue;
        const double a_in = S.acc[0], a_pr = S.acc[1], a_sx = S.acc[2], a_c = S.acc[3], a_e = S.acc[4];
        const double sn_direct = S.sn;
#pragma unroll
        for (int j = 0; j < 5; ++j) S.acc[j] = 0.0;
        S.sn = 0.0;
        const double kk = 2.0 * S.c / (1.0 - S.c);
        if (a_c == 0.0) {
            // nothing above the threshold: the state is final before this sweep
            S.stop_after = t - 1;
            S.last_bound = kk * (ordered ? sn_direct : a_in) / S.sx;
            continue;
        }
        const double sn = ordered ? sn_direct : a_in + S.c * a_pr;
        const double sx = S.sx + S.c * a_sx;
        const double bound = kk * sn / sx;
        S.sx = sx;
        S.sweeps = t + 1;
        S.tot_pushes += (unsigned long long)a_c;
        S.tot_edges += (unsigned long long)a_e;
        S.last_bound = bound;
        edges += a_e;
        live += S.m_nn;
        if (stop_l1 && bound <= tol) {
            S.stop_after = t;
        } else {
            running += 1.0;
            bmax = fmax(bmax, bound);
        }
    }
    __shared__ double s0[kDecideThreads / W], s1[kDecideThreads / W], s2[kDecideThreads / W],
        s3[kDecideThreads / W];
    edges = wave_sum(edges);
    running = wave_sum(running);
    live = wave_sum(live);
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, o, W));
    if (lane_id() == 0) {
        s0[threadIdx.x / W] = edges;
        s1[threadIdx.x / W] = running;
        s2[threadIdx.x / W] = bmax;
        s3[threadIdx.x / W] = live;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double e = 0.0, r = 0.0, b = 0.0, lv = 0.0;
    for (int j = 0; j < kDecideThreads / W; ++j) {
        e += s0[j];
        r += s1[j];
        b = fmax(b, s2[j]);
        lv += s3[j];
    }
    const unsigned long long ae = (unsigned long long)e;
    const double gather = lv * live_frac;  // in-edges a gather of the live graphs reads this sweep
    const int pull = force == 1 ? 0 : (force == 2 ? 1 : (e >= kScatterShare * gather + 1.0 ? 1 : 0));
    ctl->use_pull = pull;
    ctl->sweeps = t + 1;
    ctl->pull_sweeps += pull;
    ctl->tot_edges += ae;
    ctl->tot_traversed += pull ? (unsigned long long)gather : ae;
    ctl->last_bound = b;
    if (r == 0.0) ctl->stop_after = t;  // this sweep's scatter is the last
}

// IFP2 phase 2 inputs: w2_u = c_g z_u / deg(u) with z = pibar + h, and the
// initial mass h0 = 1 of every dangling vertex.
template <typename T>
__global__ void k_set_phase2_prep(int64_t n, int32_t nN, const SetG *gs, const int32_t *offN, int32_t k,
                                  const T *h, const double *pibar, const int32_t *deg, double *w2, double *xD) {
    GraphCursor cur{offN, k};
    double c = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (i < nN) {
            if (cur.advance(i)) c = gs[cur.g].c;
            w2[i] = c * (pibar[i] + (double)h[i]) / (double)deg[i];
        } else {
            xD[i - nN] = 1.0;
        }
    }
}

// Per-graph sums of x (fin_sum) and of the residual left on non-dangling
// vertices (fin_sn) over one region: region 0 = non-dangling positions
// [0, nN) with x = pibar + h, region 1 = dangling positions with x = xD.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_final_sum(int region, int64_t len, SetG *gs, const int32_t *off,
                                                          int32_t k, const T *h, const double *pibar,
                                                          const double *xD) {
    int64_t lo, hi;
    block_range(len, lo, hi);
    if (lo >= hi) return;
    __shared__ double s_acc[kLG * 2];
    for (int j = threadIdx.x; j < kLG * 2; j += kBlock) s_acc[j] = 0.0;
    __syncthreads();
    SegAcc<2> sa{s_acc, gs, (int)(offsetof(SetG, fin_sum) / sizeof(double)), graph_of(off, k, lo)};
    GraphCursor cur{off, k};
    double a[2] = {0.0, 0.0};
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        if (cur.g >= 0 && i >= cur.end) {
            sa.add(cur.g, a);
            a[0] = a[1] = 0.0;
        }
        cur.advance(i);
        if (region == 0) {
            const double hv = (double)h[i];
            a[0] += pibar[i] + hv;
            a[1] += hv;
        } else {
            a[0] += xD[i];
        }
    }
    if (cur.g >= 0) sa.add(cur.g, a);
    __syncthreads();
    sa.flush(graph_of(off, k, hi - 1));
}

// pi[perm[i]] = x_i / fin_sum of i's graph (the normalisation of Eq. 4)
template <typename T>
__global__ void k_set_final_write(int64_t n, int32_t nN, const SetG *gs, const int32_t *offN, const int32_t *offD,
                                  int32_t k, const int32_t *perm, const T *h, const double *pibar, const double *xD,
                                  double *out) {
    GraphCursor cn{offN, k}, cd{offD, k};
    double inv = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double x;
        if (i < nN) {
            if (cn.advance(i)) inv = 1.0 / gs[cn.g].fin_sum;
            x = pibar[i] + (double)h[i];
        } else {
            if (cd.advance(i - nN)) inv = 1.0 / gs[cd.g].fin_sum;
            x = xD[i - nN];
        }
        out[perm[i]] = x * inv;
    }
}

// ---- launchers
#define PRK_LAUNCH(kern, grid, ...)                                  \
    do {                                                             \
        hipLaunchKernelGGL((kern), dim3(grid), dim3(kBlock), 0, s,   \
                           __VA_ARGS__);                             \
        return hipGetLastError();                                    \
    } while (0)

template <typename T>
hipError_t launch_set_init(int64_t n, int32_t nN, T *h, double *pibar, hipStream_t s) {
    PRK_LAUNCH(k_set_init<T>, grid_for(n, 4, 4096), n, nN, h, pibar);
}

template <typename T>
hipError_t launch_set_reserve(int t, const Ctl *ctl, SetG *gs, const int32_t *pos_off, const int32_t *base,
                              int32_t k, int32_t len, T *h, T *w, double *pibar, const int32_t *deg,
                              const uint32_t *rp_nn, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    PRK_LAUNCH(k_set_reserve<T>, grid_for(len, 4, 2048), t, ctl, gs, pos_off, base, k, len, h, w, pibar, deg, rp_nn);
}

template <typename T>
hipError_t launch_set_sum_h(int t, const Ctl *ctl, SetG *gs, const int32_t *offN, int32_t k, int32_t nN,
                            const T *h, hipStream_t s) {
    if (nN <= 0) return hipSuccess;
    PRK_LAUNCH(k_set_sum_h<T>, grid_for(nN, 8, 2048), t, ctl, gs, offN, k, nN, h);
}

hipError_t launch_set_tile_graphs(const MPPlan &p, const int32_t *offN, int32_t k, uint2 *out, hipStream_t s) {
    if (p.blocks == 0 || p.R == 0) return hipSuccess;
    PRK_LAUNCH(k_set_tile_graphs, grid_for(p.blocks, 1, 4096), (const uint2 *)p.plan, p.blocks, p.R, offN, k, out);
}

hipError_t launch_set_decide(int t, Ctl *ctl, SetG *gs, int32_t k, int stop_l1, double tol, double live_frac,
                             int force, int ordered, hipStream_t s) {
    hipLaunchKernelGGL(k_set_decide, dim3(1), dim3(kDecideThreads), 0, s, t, ctl, gs, k, stop_l1, tol, live_frac,
                       force, ordered);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_set_phase2_prep(int64_t n, int32_t nN, const SetG *gs, const int32_t *offN, int32_t k,
                                  const T *h, const double *pibar, const int32_t *deg, double *w2, double *xD,
                                  hipStream_t s) {
    PRK_LAUNCH(k_set_phase2_prep<T>, grid_for(n, 4, 4096), n, nN, gs, offN, k, h, pibar, deg, w2, xD);
}

template <typename T>
hipError_t launch_set_final(int64_t n, int32_t nN, SetG *gs, const int32_t *offN, const int32_t *offD, int32_t k,
                            const int32_t *perm, const T *h, const double *pibar, const double *xD, double *out,
                            hipStream_t s) {
    hipError_t e = hipSuccess;
    if (nN > 0) {
        hipLaunchKernelGGL(k_set_final_sum<T>, dim3(grid_for(nN, 4, 2048)), dim3(kBlock), 0, s, 0, (int64_t)nN,
                           gs, offN, k, h, pibar, xD);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n > nN) {
        hipLaunchKernelGGL(k_set_final_sum<T>, dim3(grid_for(n - nN, 4, 2048)), dim3(kBlock), 0, s, 1,
                           (int64_t)(n - nN), gs, offD, k, h, pibar, xD);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    PRK_LAUNCH(k_set_final_write<T>, grid_for(n, 4, 4096), n, nN, gs, offN, offD, k, perm, h, pibar, xD, out);
}

#define PRK_SET_INST(T)                                                                                              \
    template hipError_t launch_set_init<T>(int64_t, int32_t, T *, double *, hipStream_t);                            \
    template hipError_t launch_set_reserve<T>(int, const Ctl *, SetG *, const int32_t *, const int32_t *,            \
                                              int32_t, int32_t, T *, T *, double *, const int32_t *,                 \
                                              const uint32_t *, hipStream_t);                                        \
    template hipError_t launch_set_sum_h<T>(int, const Ctl *, SetG *, const int32_t *, int32_t, int32_t,             \
                                            const T *, hipStream_t);                                                 \
    template hipError_t launch_set_phase2_prep<T>(int64_t, int32_t, const SetG *, const int32_t *, int32_t,          \
                                                  const T *, const double *, const int32_t *, double *, double *,    \
                                                  hipStream_t);                                                      \
    template hipError_t launch_set_final<T>(int64_t, int32_t, SetG *, const int32_t *, const int32_t *, int32_t,     \
                                            const int32_t *, const T *, const double *, const double *, double *,    \
                                            hipStream_t);
PRK_SET_INST(float)
PRK_SET_INST(double)

}  // namespace prk
