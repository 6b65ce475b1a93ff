// pr_device.h -- device helpers shared by the kernel translation units of libpr.so:
// wave64 reductions and scans, agent-scope atomics, launch sizing.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "pr_internal.h"

namespace prk {
namespace {

constexpr int W = 64;  // wavefront size on CDNA

__device__ __forceinline__ int lane_id() { return threadIdx.x & (W - 1); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// inclusive scan across one wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
        uint32_t u = __shfl_up(v, o, W);
        if (l >= o) v += u;
    }
    return v;
}

// block-wide sum, result valid in thread 0; sbuf holds kBlock / W entries
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sbuf) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) sbuf[threadIdx.x / W] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kBlock / W; ++k) r += sbuf[k];
    }
    return r;
}

__device__ __forceinline__ void atomic_add_f64(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic second stage of a two-stage reduction: one workgroup sums
// nb per-workgroup partials in a fixed order.  Result valid in thread 0.
__device__ __forceinline__ double reduce_partials(const double *part, int nb, double *sbuf) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += part[b];
    return block_sum(s, sbuf);
}

inline int grid_for(int64_t work, int per_thread, int cap) {
    int64_t b = (work + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Streaming loads (edge ids, row offsets), read once per sweep.  Plain cached loads:
// non-temporal loads were measured to make every gather 1.5-1.8x slower.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return *p;
}

// Workgroups of a tile-looping sweep kernel: exactly as many as can be resident
// at once on the device (CUs x workgroups per CU for this kernel's LDS and
// registers), so every workgroup runs from the start and the tiles are spread
// evenly; a launch whose sweep mode is not selected costs one short wave of
// workgroups.
template <typename K>
int resident_grid(K kern) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess || per_cu <= 0)
        per_cu = 4;
    return cus * per_cu;
}

}  // namespace
}  // namespace prk
