/* adg_peaks.h — measured device ceilings for the roofline of the ADG kernels.
 *
 * Two self-contained kernels give the MI355X ceilings that the stage kernels
 * are compared with next to the published ones: a streaming device copy (the
 * HBM bandwidth a kernel can actually draw: read + write bytes per second) and
 * chains of independent FP64 fused multiply-adds (the FP64 vector rate).  They
 * compute nothing of the method.
 *
 * All calls enqueue on the given HIP stream, synchronise before returning and
 * return 0, or a negative HIP error code.  Buffers are caller-owned device
 * memory.
 */
#pragma once
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` bytes (a multiple of 16) from src to dst n_reps times after one
   untimed copy; *gbs receives 2 * bytes / (mean time per copy) in GB/s. */
int32_t adg_peak_copy(const void *src, void *dst, size_t bytes, int32_t n_reps, void *hip_stream, double *gbs);

/* Size of the output buffer adg_peak_fp64 needs (one double per thread). */
size_t adg_peak_fp64_out_bytes(void);

/* Eight independent chains of 4096 FMAs per thread over a grid of eight wavefronts
   per SIMD, n_reps timed launches after one untimed one; *tflops receives
   2 * (FMAs per launch) / (mean time per launch) in TFLOP/s.  out receives
   each thread's sum (adg_peak_fp64_out_bytes() bytes). */
int32_t adg_peak_fp64(void *out, int32_t n_reps, void *hip_stream, double *tflops);

/* FP64 fused multiply-adds one launch of adg_peak_fp64's kernel performs, counted per
   lane: a kernel of known FP64 work, by which the per-kernel FP64 instruction counters
   of a profiler can be read as operations. */
double adg_peak_fp64_fmas(void);

#ifdef __cplusplus
}
#endif
