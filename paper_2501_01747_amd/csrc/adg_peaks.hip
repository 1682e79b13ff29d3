// Ceiling probes for the roofline: a streaming copy and FP64 FMA chains.
#include <hip/hip_runtime.h>

#include "adg_peaks.h"

namespace {

constexpr int kCopyBlock = 256;
constexpr int kCopyBlocks = 256 * 64;    // 64 workgroups per CU, grid-stride
constexpr int kFmaBlock = 256;
constexpr int kFmaBlocks = 256 * 8;      // 8 wavefronts per SIMD
constexpr int kFmaIters = 4096;
constexpr int kFmaChains = 8;

typedef double dv2 __attribute__((ext_vector_type(2)));

// Grid-stride copy of n 16-byte words, four loads in flight per thread, non-temporal
// (the copied data is not read again; of the variants measured, this one drew the most
// bandwidth).
__global__ __launch_bounds__(kCopyBlock) void copy_kernel(const dv2 *__restrict__ src, dv2 *__restrict__ dst,
                                                          size_t n) {
  const size_t stride = (size_t)gridDim.x * kCopyBlock;
  size_t i = (size_t)blockIdx.x * kCopyBlock + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    dv2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// kFmaChains independent chains a <- a * x + y per thread.
__global__ __launch_bounds__(kFmaBlock) void fma_kernel(double *__restrict__ out, double x, double y) {
  const int t = blockIdx.x * kFmaBlock + threadIdx.x;
  double a[kFmaChains];
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) a[c] = 1e-3 * (t + c);
  for (int it = 0; it < kFmaIters; ++it) {
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) a[c] = fma(a[c], x, y);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) s += a[c];
  out[t] = s;
}

template <class F>
int32_t timed(hipStream_t st, int32_t n_reps, F launch, double *ms_mean) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return -(int32_t)e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) { (void)hipEventDestroy(e0); return -(int32_t)e; }
  launch();
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < n_reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return -(int32_t)e;
  *ms_mean = ms / n_reps;
  return 0;
}

}  // namespace

extern "C" int32_t adg_peak_copy(const void *src, void *dst, size_t bytes, int32_t n_reps, void *hip_stream,
                                 double *gbs) {
  if (!src || !dst || !gbs || n_reps < 1 || bytes == 0 || bytes % 16) return -(int32_t)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = bytes / 16;
  double ms = 0.0;
  const int32_t rc = timed(st, n_reps, [&] {
    hipLaunchKernelGGL(copy_kernel, dim3(kCopyBlocks), dim3(kCopyBlock), 0, st, (const dv2 *)src, (dv2 *)dst, n);
  }, &ms);
  if (rc) return rc;
  *gbs = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
  return 0;
}

extern "C" size_t adg_peak_fp64_out_bytes(void) { return sizeof(double) * (size_t)kFmaBlocks * kFmaBlock; }

extern "C" double adg_peak_fp64_fmas(void) { return (double)kFmaBlocks * kFmaBlock * kFmaIters * kFmaChains; }

extern "C" int32_t adg_peak_fp64(void *out, int32_t n_reps, void *hip_stream, double *tflops) {
  if (!out || !tflops || n_reps < 1) return -(int32_t)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)hip_stream;
  double ms = 0.0;
  const int32_t rc = timed(st, n_reps, [&] {
    hipLaunchKernelGGL(fma_kernel, dim3(kFmaBlocks), dim3(kFmaBlock), 0, st, (double *)out, 0.999999, 1e-7);
  }, &ms);
  if (rc) return rc;
  *tflops = 2.0 * adg_peak_fp64_fmas() / (ms * 1e-3) / 1e12;
  return 0;
}
