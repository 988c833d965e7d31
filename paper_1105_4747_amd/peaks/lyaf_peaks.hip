// lyaf_peaks.hip -- microbenchmarks of the device rates that bound the
// optical-depth kernels: independent FP32 FMAs, independent exp2 (the
// transcendental unit alone), exp2 issued beside a growing number of FMAs (does
// the transcendental work overlap the other VALU work?), the per-pair
// arithmetic of the tau sum with and without its exp2, and a streaming copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lyaf_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMixN = LYAF_PEAKS_MIX_N;
constexpr int kMixNV[kMixN] = {0, 1, 2, 3, 4, 6};
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

// Four independent exp2 chains per lane (x <- exp2(-x) stays in (1/2, 1)).
__global__ __launch_bounds__(kThreads) void peak_exp_kernel(float *out) {
  float x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = 0.5f + threadIdx.x * 1e-4f + 0.1f * c;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
  }
  const float s = (x[0] + x[1]) + (x[2] + x[3]);
  if (s == 1234.5f) out[threadIdx.x] = s;
}

// Per iteration: the four exp2 chains above and 4 NV independent FMA chains.
// With an overlapping transcendental unit the time is the larger of the two
// streams; without, their sum.
template <int NV>
__global__ __launch_bounds__(kThreads) void peak_mix_kernel(float *out, float a, float b) {
  float x[4], y[4 * NV > 0 ? 4 * NV : 1];
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = 0.5f + threadIdx.x * 1e-4f + 0.1f * c;
#pragma unroll
  for (int c = 0; c < 4 * NV; ++c) y[c] = threadIdx.x * 1e-4f + c;
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[c] = __builtin_amdgcn_exp2f(-x[c]);
#pragma unroll
      for (int v = 0; v < NV; ++v) y[c * NV + v] = __builtin_fmaf(y[c * NV + v], a, b);
    }
  }
  float s = (x[0] + x[1]) + (x[2] + x[3]);
#pragma unroll
  for (int c = 0; c < 4 * NV; ++c) s += y[c];
  if (s == 1234.5f) out[threadIdx.x] = s;
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
  double t_fma = 0, t_exp = 0, t_noexp = 0, t_copy = 0, t_trans = 0;
  double t_mix[kMixN] = {};
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
  if (e == hipSuccess)
    e = time_launch(
        [&] { hipLaunchKernelGGL(peak_exp_kernel, dim3(blocks), dim3(kThreads), 0, st,
                                 scratch); },
        st, 3, &t_trans);
  // exp2 beside 4 NV FMA chains, NV = kMixNV[k]
  auto mix = [&](auto nv, double *t) {
    constexpr int NV = decltype(nv)::value;
    return time_launch(
        [&] { hipLaunchKernelGGL(peak_mix_kernel<NV>, dim3(blocks), dim3(kThreads), 0, st,
                                 scratch, 0.999f, 1e-3f); },
        st, 3, t);
  };
  if (e == hipSuccess) e = mix(std::integral_constant<int, 0>{}, &t_mix[0]);
  if (e == hipSuccess) e = mix(std::integral_constant<int, 1>{}, &t_mix[1]);
  if (e == hipSuccess) e = mix(std::integral_constant<int, 2>{}, &t_mix[2]);
  if (e == hipSuccess) e = mix(std::integral_constant<int, 3>{}, &t_mix[3]);
  if (e == hipSuccess) e = mix(std::integral_constant<int, 4>{}, &t_mix[4]);
  if (e == hipSuccess) e = mix(std::integral_constant<int, 6>{}, &t_mix[5]);
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
  const double exps = lanes * kIters * 4;
  out->fma_lane_ops_per_s = fma_ops / t_fma;
  out->trans_lane_ops_per_s = exps / t_trans;
  out->pair_per_s_exp = pairs / t_exp;
  out->pair_per_s_noexp = pairs / t_noexp;
  out->c_valu_s = t_fma / fma_ops;
  out->c_exp_s = (t_exp - t_noexp) / pairs;
  // every pair of the direct form issues its own exp2 and at least three other
  // VALU operations (t_k, its square, the accumulate); with the two units
  // overlapping, the slower stream bounds the rate
  out->pair_peak_per_s = std::min(out->fma_lane_ops_per_s / 3.0, out->trans_lane_ops_per_s);
  for (int k = 0; k < kMixN; ++k) {
    out->mix_fma_per_exp[k] = 1.0 * kMixNV[k];
    out->mix_exp_per_s[k] = exps / t_mix[k];
  }
  out->copy_bytes_per_s = 2.0 * (double)n4 * sizeof(float4) / t_copy;
  out->compute_units = prop.multiProcessorCount;
  out->clock_khz = prop.clockRate;
  return 0;
}
