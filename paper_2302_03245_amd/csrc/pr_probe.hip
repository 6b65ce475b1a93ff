// pr_probe.hip -- measurement kernels used by the benchmark to place the solver
// kernels against the chip: a streaming copy (achievable HBM bandwidth and the
// calibration of the hardware byte counters), and index-driven random gather
// and FP32 atomic scatter (the two ways a sweep touches the residual vector).
#include <hip/hip_runtime.h>

#include "../../include/pr_probe.h"

namespace {

constexpr int kB = 256;

__global__ __launch_bounds__(kB) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n4) {
    for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kB) dst[i] = src[i];
}

__global__ __launch_bounds__(kB) void k_gather(const float *__restrict__ w, const int32_t *__restrict__ idx,
                                               int64_t m, float *__restrict__ out) {
    float acc = 0.f;
    for (int64_t e = blockIdx.x * (int64_t)kB + threadIdx.x; e < m; e += (int64_t)gridDim.x * kB) acc += w[idx[e]];
    out[blockIdx.x * (int64_t)kB + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kB) void k_scatter(float *__restrict__ h, const int32_t *__restrict__ idx, int64_t m,
                                                float v) {
    for (int64_t e = blockIdx.x * (int64_t)kB + threadIdx.x; e < m; e += (int64_t)gridDim.x * kB)
        atomicAdd(h + idx[e], v);
}

int grid(int64_t work, int cap) {
    int64_t b = (work + kB * 4 - 1) / (kB * 4);
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

template <typename F>
int timed(void *stream, int reps, double *seconds, F launch) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -3;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -3;
    }
    launch(s);  // warm-up
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) launch(s);
    (void)hipEventRecord(b, s);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (seconds) *seconds = ms * 1e-3 / (reps > 0 ? reps : 1);
    return e == hipSuccess ? 0 : -3;
}

}  // namespace

extern "C" {

int pr_probe_copy(const void *src, void *dst, int64_t bytes, int reps, void *stream, double *seconds) {
    if (!src || !dst || bytes <= 0 || (bytes % 16) || reps < 1) return -1;
    const int64_t n4 = bytes / 16;
    return timed(stream, reps, seconds, [&](hipStream_t s) {
        hipLaunchKernelGGL(k_copy, dim3(grid(n4, 65536)), dim3(kB), 0, s, (const float4 *)src, (float4 *)dst, n4);
    });
}

int pr_probe_gather(const float *w, const int32_t *idx, int64_t m, float *out, int64_t out_len, int reps,
                    void *stream, double *seconds) {
    if (!w || !idx || !out || m <= 0 || reps < 1) return -1;
    const int g = grid(m, 16384);
    if (out_len < (int64_t)g * kB) return -1;
    return timed(stream, reps, seconds, [&](hipStream_t s) {
        hipLaunchKernelGGL(k_gather, dim3(g), dim3(kB), 0, s, w, idx, m, out);
    });
}

int pr_probe_scatter(float *h, const int32_t *idx, int64_t m, float v, int reps, void *stream, double *seconds) {
    if (!h || !idx || m <= 0 || reps < 1) return -1;
    return timed(stream, reps, seconds, [&](hipStream_t s) {
        hipLaunchKernelGGL(k_scatter, dim3(grid(m, 16384)), dim3(kB), 0, s, h, idx, m, v);
    });
}

int64_t pr_probe_gather_out_len(int64_t m) { return (int64_t)grid(m, 16384) * kB; }

}  // extern "C"
