// pr_sort.hip -- upload-time ordering of the in-edge lists: every target row's
// sources sorted by (device) id.  A gather instruction covers 64 consecutive
// in-edges; with sorted rows those of a long row span a narrow range of source
// ids (the high-degree sources come first in the vertex order), so they touch
// fewer distinct cache lines; the order also makes the gathers deterministic.
#include <hipcub/hipcub.hpp>

#include "pr_device.h"
#include "pr_internal.h"

namespace prk {
namespace {

// one wave per target row: key = row << 32 | source
__global__ void k_row_keys(int64_t R, const uint32_t *in_ptr, const int32_t *in_src, unsigned long long *keys) {
    const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / W;
    const int64_t nwaves = (int64_t)gridDim.x * kBlock / W;
    for (int64_t r = wave; r < R; r += nwaves)
        for (uint32_t e = in_ptr[r] + lane_id(); e < in_ptr[r + 1]; e += W)
            keys[e] = ((unsigned long long)r << 32) | (uint32_t)in_src[e];
}

__global__ void k_keys_to_src(int64_t m, const unsigned long long *keys, int32_t *in_src) {
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < m; e += (int64_t)gridDim.x * kBlock)
        in_src[e] = (int32_t)(uint32_t)(keys[e] & 0xffffffffull);
}

}  // namespace

hipError_t sort_in_lists(int64_t n, int64_t m, const uint32_t *in_ptr, int32_t *in_src, hipStream_t s) {
    if (m <= 1) return hipSuccess;
    int bits = 1;
    while (((int64_t)1 << bits) < n) ++bits;
    unsigned long long *k0 = nullptr, *k1 = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipMalloc((void **)&k0, sizeof(unsigned long long) * (size_t)m);
    if (e == hipSuccess) e = hipMalloc((void **)&k1, sizeof(unsigned long long) * (size_t)m);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_row_keys, dim3(grid_for(n * W, 1, 16384)), dim3(kBlock), 0, s, n, in_ptr, in_src, k0);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, k0, k1, (int)m, 0, 32 + bits, s);
    if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 1));
    if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, k0, k1, (int)m, 0, 32 + bits, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_keys_to_src, dim3(grid_for(m, 4, 16384)), dim3(kBlock), 0, s, m,
                           (const unsigned long long *)k1, in_src);
        e = hipGetLastError();
    }
    // the temporaries are freed once the stream has used them
    hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (tmp) (void)hipFree(tmp);
    if (k1) (void)hipFree(k1);
    if (k0) (void)hipFree(k0);
    return e;
}

}  // namespace prk
