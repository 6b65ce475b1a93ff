// pr_warm.hip -- kernels of the warm start (include/pr_warm.h): a forward-push
// state (reserve pibar and residual h over all vertices, original ids) moved
// into a solve's device order and back, and carried over a change of the graph.
//
// The state obeys x = pibar + (I - cP)^{-1} h, x the exact unnormalised vector
// (Eq. 4 with this p), because every push keeps pibar + (I - cP)^{-1} h fixed.
// For a changed matrix P' the same reserve with h' = h + c (P' - P) pibar
// satisfies it again, and only the columns of sources whose out-edges changed
// contribute.  IFP2's phase 1 does not push into dangling vertices; its state is
// exported in the equivalent form where the mass taken so far has also reached
// them: h_d += c sum over in-edges u -> d of (taken mass of u) / deg(u).
#include <hip/hip_runtime.h>

#include "pr_device.h"
#include "pr_internal.h"

namespace prk {
namespace {

// device order <- state (original ids): non-dangling pibar, pibar0 (copy), h; dangling:
// xD0 = pibar + h (the start of phase 2), hD0 = h; per-workgroup mass partials
template <typename T>
__global__ __launch_bounds__(kBlock) void k_warm_import(int64_t n, int32_t nN, const int32_t *perm,
                                                        const double *st_pibar, const double *st_h, T *h,
                                                        double *pibar, double *pibar0, double *xD0, double *hD0,
                                                        double *part) {
    double mass = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t o = perm[i];
        const double pb = st_pibar[o], hv = st_h[o];
        mass += pb + hv;
        h[i] = (T)hv;
        if (i < nN) {
            pibar[i] = pb;
            pibar0[i] = pb;
        } else {
            xD0[i - nN] = pb + hv;
            hD0[i - nN] = hv;
        }
    }
    __shared__ double sd[kBlock / W];
    mass = block_sum(mass, sd);
    if (threadIdx.x == 0) part[blockIdx.x] = mass;
}

// total mass of the imported state, and the signed form of the stop rule
__global__ __launch_bounds__(kBlock) void k_warm_mass(Ctl *ctl, int nb, const double *part) {
    __shared__ double sd[kBlock / W];
    const double m = reduce_partials(part, nb, sd);
    if (threadIdx.x == 0) {
        ctl->sx = m;
        ctl->signed_res = 1;
    }
}

// phase-2 inputs of a resumed IFP2 solve: w2 = c (taken this solve + residual) / deg
// for the folded result; w3 = c (taken this solve) / deg for the exported state
template <typename T>
__global__ void k_warm_phase2_prep(int32_t nN, int32_t nD, const T *h, const double *pibar, const double *pibar0,
                                   const int32_t *deg, double c, const double *xD0, const double *hD0, double *w2,
                                   double *w3, double *xD, double *hDn) {
    const int64_t tot = (int64_t)nN + nD;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < tot; i += (int64_t)gridDim.x * kBlock) {
        if (i < nN) {
            const double taken = pibar[i] - pibar0[i];
            w2[i] = c * (taken + (double)h[i]) / (double)deg[i];
            w3[i] = c * taken / (double)deg[i];
        } else {
            xD[i - nN] = xD0[i - nN];
            hDn[i - nN] = hD0[i - nN];
        }
    }
}

// state (original ids) <- device order: non-dangling pibar and h, dangling h with the
// mass taken during the solve pushed in (their pibar is unchanged)
template <typename T>
__global__ void k_warm_export(int64_t n, int32_t nN, const int32_t *perm, const T *h, const double *pibar,
                              const double *hDn, double *st_pibar, double *st_h) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t o = perm[i];
        if (i < nN) {
            st_pibar[o] = pibar[i];
            st_h[o] = (double)h[i];
        } else {
            st_h[o] = hDn[i - nN];
        }
    }
}

// h += c (P_new - P_old) pibar for the listed sources (all when src is null): one wave
// per source removes c pibar_u / deg_old(u) from every old out-neighbour and adds
// c pibar_u / deg_new(u) to every new one
struct GView {
    const int32_t *newid, *perm, *deg;
    const uint32_t *rp_nn, *rp_nd;
    const int32_t *col_nn, *col_nd;
    int32_t nN;
};

__device__ __forceinline__ void spread(const GView &g, int32_t u, double f, double *st_h) {
    const int32_t ud = g.newid[u];
    if (ud >= g.nN) return;  // no out-edges
    const double a = f / (double)g.deg[ud];
    for (uint32_t e = g.rp_nn[ud] + lane_id(); e < g.rp_nn[ud + 1]; e += W)
        atomic_add_f64(st_h + g.perm[g.col_nn[e]], a);
    for (uint32_t e = g.rp_nd[ud] + lane_id(); e < g.rp_nd[ud + 1]; e += W)
        atomic_add_f64(st_h + g.perm[g.col_nd[e]], a);
}

__global__ __launch_bounds__(kBlock) void k_state_update(const int32_t *src, int64_t count, GView go, GView gn,
                                                         double c, const double *st_pibar, double *st_h) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t q = wave; q < count; q += nwaves) {
        const int32_t u = src ? src[q] : (int32_t)q;
        const double pb = st_pibar[u];
        if (pb == 0.0) continue;
        spread(go, u, -c * pb, st_h);
        spread(gn, u, c * pb, st_h);
    }
}

GView view_of(const Graph &G) {
    GView v;
    v.newid = G.newid;
    v.perm = G.perm;
    v.deg = G.deg;
    v.rp_nn = G.rp_nn;
    v.rp_nd = G.rp_nd;
    v.col_nn = G.col_nn;
    v.col_nd = G.col_nd;
    v.nN = G.nN;
    return v;
}

}  // namespace

template <typename T>
hipError_t launch_warm_import(Ctl *ctl, int64_t n, int32_t nN, const int32_t *perm, const double *st_pibar,
                              const double *st_h, T *h, double *pibar, double *pibar0, double *xD0, double *hD0,
                              double *part, hipStream_t s) {
    const int nb = grid_for(n, 4, kRedBlocks);
    hipLaunchKernelGGL(k_warm_import<T>, dim3(nb), dim3(kBlock), 0, s, n, nN, perm, st_pibar, st_h, h, pibar,
                       pibar0, xD0, hD0, part);
    hipLaunchKernelGGL(k_warm_mass, dim3(1), dim3(kBlock), 0, s, ctl, nb, (const double *)part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_phase2_prep(int32_t nN, int32_t nD, const T *h, const double *pibar, const double *pibar0,
                                   const int32_t *deg, double c, const double *xD0, const double *hD0, double *w2,
                                   double *w3, double *xD, double *hDn, hipStream_t s) {
    hipLaunchKernelGGL(k_warm_phase2_prep<T>, dim3(grid_for((int64_t)nN + nD, 4, 8192)), dim3(kBlock), 0, s, nN,
                       nD, h, pibar, pibar0, deg, c, xD0, hD0, w2, w3, xD, hDn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_export(int64_t n, int32_t nN, const int32_t *perm, const T *h, const double *pibar,
                              const double *hDn, double *st_pibar, double *st_h, hipStream_t s) {
    hipLaunchKernelGGL(k_warm_export<T>, dim3(grid_for(n, 4, 8192)), dim3(kBlock), 0, s, n, nN, perm, h, pibar,
                       hDn, st_pibar, st_h);
    return hipGetLastError();
}

hipError_t launch_state_update(const int32_t *src, int64_t count, const Graph &g_old, const Graph &g_new, double c,
                               const double *st_pibar, double *st_h, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_state_update, dim3(grid_for(count * W, 1, 16384)), dim3(kBlock), 0, s, src, count,
                       view_of(g_old), view_of(g_new), c, st_pibar, st_h);
    return hipGetLastError();
}

template hipError_t launch_warm_import<float>(Ctl *, int64_t, int32_t, const int32_t *, const double *,
                                              const double *, float *, double *, double *, double *, double *,
                                              double *, hipStream_t);
template hipError_t launch_warm_import<double>(Ctl *, int64_t, int32_t, const int32_t *, const double *,
                                               const double *, double *, double *, double *, double *, double *,
                                               double *, hipStream_t);
template hipError_t launch_warm_phase2_prep<float>(int32_t, int32_t, const float *, const double *, const double *,
                                                   const int32_t *, double, const double *, const double *,
                                                   double *, double *, double *, double *, hipStream_t);
template hipError_t launch_warm_phase2_prep<double>(int32_t, int32_t, const double *, const double *,
                                                    const double *, const int32_t *, double, const double *,
                                                    const double *, double *, double *, double *, double *,
                                                    hipStream_t);
template hipError_t launch_warm_export<float>(int64_t, int32_t, const int32_t *, const float *, const double *,
                                              const double *, double *, double *, hipStream_t);
template hipError_t launch_warm_export<double>(int64_t, int32_t, const int32_t *, const double *, const double *,
                                               const double *, double *, double *, hipStream_t);

}  // namespace prk
