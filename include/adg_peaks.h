/* adg_peaks.h: measurement kernels for the roofline of the ADER-DG kernels
 * (libadg_peaks.so).  They are not part of the method: they measure what the
 * device reaches on the two resources that bound the step, so that achieved
 * rates can be put beside both the published and the achievable peak:
 *   - vector FMA throughput (float64, float), the bound of the predictor;
 *   - HBM bandwidth of a streaming copy and triad, the bound of the corrector.
 *
 * Conventions: every pointer argument is a caller-owned device pointer; the
 * calls enqueue one kernel on `stream` and return at once (the caller times
 * them with events on that stream); the library allocates nothing.  Return
 * value 0 on success, 1 for an invalid argument (nothing is launched), 3 for
 * a launch error reported by the runtime.
 */
#ifndef ADG_PEAKS_H
#define ADG_PEAKS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dependent-FMA chains: `blocks` workgroups of 256 threads, each thread runs
 * 16 independent chains of `iters` fused multiply-adds and writes one value
 * to d_sink[blocks * 256] (double for precision 0, float for 1), so the work
 * cannot be removed.  Flops per launch = blocks * 256 * 16 * iters * 2.
 * precision: 0 = float64, 1 = float (non-packed FMA).  blocks in [1, 65536],
 * iters in [1, 1 << 20], d_sink non-null and 256-byte aligned. */
int32_t adg_peak_fma(int32_t precision, int32_t blocks, int32_t iters, void* d_sink,
                     hipStream_t stream);

/* Streaming copy d_dst[i] = d_src[i], i < n (float64), 16-byte vector
 * accesses.  Bytes moved = 16 n.  n >= 0; both pointers non-null and 16-byte
 * aligned when n > 0; the ranges must not overlap. */
int32_t adg_stream_copy(const double* d_src, double* d_dst, int64_t n, hipStream_t stream);

/* Streaming triad d_c[i] = d_a[i] + s d_b[i], i < n (float64).  Bytes moved
 * = 24 n.  Same pointer rules as adg_stream_copy. */
int32_t adg_stream_triad(const double* d_a, const double* d_b, double* d_c, double s, int64_t n,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ADG_PEAKS_H */
