// lyaf_peaks.hip -- microbenchmarks of the device rates that bound the
// optical-depth kernels: independent FP32 FMAs, the per-pair arithmetic of the
// tau sum with and without its exp2, and a streaming copy.
#include <hip/hip_runtime.h>

#include "lyaf_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kIters = 4096;
constexpr int kChains = 8;

__global__ __launch_bounds__(kThreads) void peak_fma_kernel(float *out, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 1e-4f + c;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == 1234.5f) out[threadIdx.x] = s;  // never true: keeps the work
}

// One source against four consecutive targets per iteration, as in the tau
// loop: t_k = k a + t0, e = exp2(-t_k^2), acc_k += w e.
template <bool EXP>
__global__ __launch_bounds__(kThreads) void peak_pair_kernel(float *out, float a, float w) {
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float t0 = threadIdx.x * 1e-4f;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = __builtin_fmaf((float)k, a, t0);
      const float x = -(t * t);
      const float e = EXP ? __builtin_amdgcn_exp2f(x) : x;
      acc[k] = __builtin_fmaf(w, e, acc[k]);
    }
    t0 += 1e-3f;
  }
  const float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (s == 1234.5f) out[threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void peak_copy_kernel(const float4 *__restrict__ src,
                                                             float4 *__restrict__ dst,
                                                             int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    dst[i] = src[i];
}

// Average seconds per launch of `launch` over `reps` launches after one warm-up.
template <typename F>
hipError_t time_launch(F launch, hipStream_t st, int reps, double *sec) {
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  launch();
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  *sec = (double)ms * 1e-3 / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" int lyaf_peaks_measure(lyaf_peak_rates *out, void *stream) {
  if (!out) return -1;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return -5;
  const int blocks = prop.multiProcessorCount * 8;  // eight 4-wave workgroups per CU
  const double lanes = (double)blocks * kThreads;
  float *scratch = nullptr;
  float4 *src = nullptr, *dst = nullptr;
  const int64_t n4 = (int64_t)1 << 25;  // 512 MiB per buffer
  if (hipMalloc((void **)&scratch, kThreads * sizeof(float)) != hipSuccess) return -6;
  if (hipMalloc((void **)&src, n4 * sizeof(float4)) != hipSuccess ||
      hipMalloc((void **)&dst, n4 * sizeof(float4)) != hipSuccess) {
    (void)hipFree(scratch);
    if (src) (void)hipFree(src);
    return -6;
  }
  double t_fma = 0, t_exp = 0, t_noexp = 0, t_copy = 0;
  hipError_t e = time_launch(
      [&] { hipLaunchKernelGGL(peak_fma_kernel, dim3(blocks), dim3(kThreads), 0, st, scratch,
                               0.999f, 1e-3f); },
      st, 3, &t_fma);
  if (e == hipSuccess)
    e = time_launch(
        [&] { hipLaunchKernelGGL(peak_pair_kernel<true>, dim3(blocks), dim3(kThreads), 0, st,
                                 scratch, 0.1f, 1.f); },
        st, 3, &t_exp);
  if (e == hipSuccess)
    e = time_launch(
        [&] { hipLaunchKernelGGL(peak_pair_kernel<false>, dim3(blocks), dim3(kThreads), 0, st,
                                 scratch, 0.1f, 1.f); },
        st, 3, &t_noexp);
  if (e == hipSuccess && hipMemsetAsync(src, 0, n4 * sizeof(float4), st) != hipSuccess)
    e = hipErrorUnknown;
  if (e == hipSuccess)
    e = time_launch(
        [&] { hipLaunchKernelGGL(peak_copy_kernel, dim3(prop.multiProcessorCount * 16),
                                 dim3(kThreads), 0, st, src, dst, n4); },
        st, 3, &t_copy);
  (void)hipFree(scratch);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return -5;
  const double fma_ops = lanes * kIters * kChains;
  const double pairs = lanes * kIters * 4;
  out->fma_lane_ops_per_s = fma_ops / t_fma;
  out->pair_per_s_exp = pairs / t_exp;
  out->pair_per_s_noexp = pairs / t_noexp;
  out->c_valu_s = t_fma / fma_ops;
  out->c_exp_s = (t_exp - t_noexp) / pairs;
  out->pair_peak_per_s = 1.0 / (out->c_exp_s + 4.0 * out->c_valu_s);
  out->copy_bytes_per_s = 2.0 * (double)n4 * sizeof(float4) / t_copy;
  out->compute_units = prop.multiProcessorCount;
  out->clock_khz = prop.clockRate;
  return 0;
}
