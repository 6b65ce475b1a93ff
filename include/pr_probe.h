/*
 * pr_probe.h -- measurement kernels exported by libpr.so for the benchmark.
 *
 * They bound the solver kernels from above on the same chip: the forward-push
 * sweep streams edge indices and then either scatters an FP32 add to, or
 * gathers a value from, a random entry of a residual-sized vector (the pushes
 * of Algorithms 2 and 3 as seen by memory).  All pointers are device pointers,
 * all calls run on `stream` (NULL = default stream) and return 0 on success,
 * -1 on an invalid argument, -3 on a HIP error.  *seconds receives the mean
 * duration of one launch over `reps` timed launches (after one warm-up).
 * The caller owns every buffer; idx entries must index inside w / h (the probe
 * does not check them).
 */
#ifndef PR_PROBE_H
#define PR_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0..bytes) = src[0..bytes); bytes a positive multiple of 16 */
int pr_probe_copy(const void *src, void *dst, int64_t bytes, int reps, void *stream, double *seconds);

/* per-thread sums of w[idx[e]] over e in [0, m) written to out (out_len >= pr_probe_gather_out_len(m)) */
int pr_probe_gather(const float *w, const int32_t *idx, int64_t m, float *out, int64_t out_len, int reps,
                    void *stream, double *seconds);

/* h[idx[e]] += v for e in [0, m) with hardware FP32 atomic adds */
int pr_probe_scatter(float *h, const int32_t *idx, int64_t m, float v, int reps, void *stream, double *seconds);

/* length of the out buffer pr_probe_gather needs for m indices */
int64_t pr_probe_gather_out_len(int64_t m);

#ifdef __cplusplus
}
#endif

#endif /* PR_PROBE_H */
