// lyaf_stats.hip -- flux statistics of Greig, Bolton & Wyithe (2011), Section 4:
// the flux PDF (Section 4.2) and the 1D line-of-sight flux power spectrum
// (Section 4.3).
//
// Flux PDF: 21 bins of width 0.05 centred on F = 0 .. 1; bin j holds
// 0.05 j - 0.025 <= F < 0.05 j + 0.025, decided as j = floor((F + 0.025) * 20)
// in FP64 on the exact FP32 input (one rounding after the sum, one after the
// product).  Values below, at or above the end, and NaN are counted apart.
// Each lane counts into its own LDS column (address slot * 256 + lane: every
// lane on its own bank, no atomics), each workgroup writes its 24 counts, and a
// second kernel sums them in a fixed order, so the output is exact and is
// overwritten.
//
// Power spectrum: per skewer of N pixels (a power of two, 2 .. 8192),
// delta_j = F_j / Fbar - 1 and P(k_m) = (dv / N) |sum_j delta_j e^{-2 pi i m j / N}|^2,
// m = 0 .. N/2.  One workgroup per skewer packs the N reals into M = N/2
// complex values z_j = delta_{2j} + i delta_{2j+1}, transforms them in LDS in
// FP64 (Stockham passes of radix 8, then one of radix 4 or 2 as log2 M needs,
// in place: each thread holds its butterflies' outputs in registers across a
// barrier), with twiddles read from one half-period table of the largest
// transform, exp(-2 pi i t / 4096), t < 2048, built once (cached in L1/L2; the
// table of M points is every (4096 / M)-th entry), and unpacks
// X_m = E_m + e^{-pi i m / M} O_m with E_m = (Z_m + conj Z_{M-m}) / 2 and
// O_m = (Z_m - conj Z_{M-m}) / 2i.
#include <algorithm>

#include "lyaf_fft.h"
#include "lyaf_internal.h"

namespace lyaf {
namespace {

constexpr int kPdfThreads = 256;
constexpr int kPdfSlots = 24;  // 21 bins, below, above, NaN
constexpr int kPsThreads = 256;

__device__ inline int pdf_slot(float f) {
  const double t = ((double)f + 0.025) * 20.0;
  if (t != t) return 23;      // NaN
  if (t < 0.0) return 21;     // below the first bin
  if (t >= 21.0) return 22;   // at or above the end of the last bin
  return (int)t;
}

__global__ __launch_bounds__(kPdfThreads) void flux_pdf_kernel(const float *__restrict__ F,
                                                               int64_t n,
                                                               uint32_t *__restrict__ part) {
  __shared__ uint32_t cnt[kPdfSlots * kPdfThreads];
  const int tid = threadIdx.x;
#pragma unroll
  for (int b = 0; b < kPdfSlots; ++b) cnt[b * kPdfThreads + tid] = 0;
  const int64_t stride = (int64_t)gridDim.x * kPdfThreads;
  int64_t i = (int64_t)blockIdx.x * kPdfThreads + tid;
  // four values in flight per thread; the LDS adds return nothing, so they do
  // not wait on one another (a lane's column is its own: no contention)
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float f0 = F[i], f1 = F[i + stride], f2 = F[i + 2 * stride], f3 = F[i + 3 * stride];
    atomicAdd(&cnt[pdf_slot(f0) * kPdfThreads + tid], 1u);
    atomicAdd(&cnt[pdf_slot(f1) * kPdfThreads + tid], 1u);
    atomicAdd(&cnt[pdf_slot(f2) * kPdfThreads + tid], 1u);
    atomicAdd(&cnt[pdf_slot(f3) * kPdfThreads + tid], 1u);
  }
  for (; i < n; i += stride) atomicAdd(&cnt[pdf_slot(F[i]) * kPdfThreads + tid], 1u);
  __syncthreads();
  if (tid < kPdfSlots) {
    uint32_t s = 0;  // rotated start: the 24 summing lanes read different banks
    for (int l = 0; l < kPdfThreads; ++l) s += cnt[tid * kPdfThreads + ((l + tid) & 255)];
    part[(int64_t)blockIdx.x * kPdfSlots + tid] = s;
  }
}

// Sum of the workgroups' counts (integers: exact in any order): one wave per
// slot, each lane summing a strided share with its reads in flight, then a
// shuffle reduction.
__global__ __launch_bounds__(64) void flux_pdf_sum_kernel(const uint32_t *__restrict__ part,
                                                          int blocks,
                                                          int64_t *__restrict__ counts) {
  const int slot = blockIdx.x;
  uint64_t s = 0;
  for (int g = threadIdx.x; g < blocks; g += 64) s += part[(int64_t)g * kPdfSlots + slot];
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  if (threadIdx.x == 0) counts[slot] = (int64_t)s;
}

// Twiddle table of the largest transform, exp(-2 pi i t / 4096), t < 2048; the
// table of a transform of M points is every (4096 / M)-th entry.
constexpr int kTwMax = kPsMaxN / 2;
static_assert(kTwMax == kFftTableLen, "one twiddle table serves every transform");
__global__ void twiddle_kernel(double2 *__restrict__ T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kTwMax / 2) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)kTwMax, &sn, &cs);
    T[t] = make_double2(cs, sn);
  }
}

__global__ __launch_bounds__(kPsThreads) void flux_power_kernel(
    const float *__restrict__ F, const int64_t *__restrict__ offsets,
    const int64_t *__restrict__ mode_off, const float *__restrict__ dv, double inv_mean,
    const double2 *__restrict__ Tg, float *__restrict__ P, uint32_t *status) {
  extern __shared__ double2 lds_ps[];
  const int64_t s = blockIdx.x;
  const int64_t off = offsets[s];
  const int N = (int)(offsets[s + 1] - off);  // a power of two, 2 .. 8192 (host-checked)
  const int M = N / 2;
  const double dvs = (double)dv[s];
  if (!(dvs > 0.0) || !isfinite(dvs)) {
    if (threadIdx.x == 0) atomicOr(status, LYAF_STATUS_DOMAIN);
    return;
  }
  double2 *buf = lds_ps;
  const float *f = F + off;
  const auto put = [&](int j, float2 v) {
    buf[j] = make_double2(__builtin_fma((double)v.x, inv_mean, -1.0),
                          __builtin_fma((double)v.y, inv_mean, -1.0));
  };
  if ((reinterpret_cast<uintptr_t>(f) & 7u) == 0) {
    // pairs of values as float2, four reads in flight per thread
    const float2 *f2 = reinterpret_cast<const float2 *>(f);
    int j = threadIdx.x;
    for (; j + 3 * kPsThreads < M; j += 4 * kPsThreads) {
      float2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = f2[j + u * kPsThreads];
#pragma unroll
      for (int u = 0; u < 4; ++u) put(j + u * kPsThreads, v[u]);
    }
    for (; j < M; j += kPsThreads) put(j, f2[j]);
  } else {
    for (int j = threadIdx.x; j < M; j += kPsThreads) put(j, make_float2(f[2 * j], f[2 * j + 1]));
  }
  __syncthreads();
  fft_batch<kPsThreads, kPsMaxN / 2>(buf, Tg, M, 0);

  // unpack the real spectrum: X_m = E_m + e^{-pi i m / M} O_m, m = 0 .. M
  double s1, c1;
  sincospi(-1.0 / (double)M, &s1, &c1);
  const double2 half_step = make_double2(c1, s1);
  const double scale = dvs / (double)N;
  float *out = P + mode_off[s];
  const auto mode = [&](int m, double2 t) {  // t: table entry (m >> 1) of this transform
    const double2 zm = buf[m == M ? 0 : m];
    const double2 zr = buf[m == 0 ? 0 : M - m];
    const double2 zc = make_double2(zr.x, -zr.y);
    const double2 E = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
    const double2 d = csub(zm, zc);
    const double2 O = make_double2(0.5 * d.y, -0.5 * d.x);  // d / 2i
    double2 tw;
    if (m == M)
      tw = make_double2(-1.0, 0.0);
    else if ((m & 1) == 0)
      tw = t;
    else
      tw = cmul(t, half_step);
    const double2 X = cadd(E, cmul(tw, O));
    out[m] = (float)(scale * __builtin_fma(X.x, X.x, X.y * X.y));
  };
  // table reads of four modes in flight per thread (entry 0 stands in at m = M)
  const auto entry = [&](int m) { return Tg[m == M ? 0 : (m >> 1) * (kTwMax / M)]; };
  int m = threadIdx.x;
  for (; m + 3 * kPsThreads <= M; m += 4 * kPsThreads) {
    double2 t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = entry(m + u * kPsThreads);
#pragma unroll
    for (int u = 0; u < 4; ++u) mode(m + u * kPsThreads, t[u]);
  }
  for (; m <= M; m += kPsThreads) mode(m, entry(m));
}

}  // namespace

int pdf_blocks(int64_t n) {
  const int64_t per_block = (int64_t)kPdfThreads * 16;
  return (int)std::max<int64_t>(1, std::min<int64_t>(kPdfMaxBlocks, (n + per_block - 1) / per_block));
}

hipError_t launch_flux_pdf(int64_t n, const float *F, uint32_t *part, int64_t *counts,
                           hipStream_t st) {
  const int blocks = pdf_blocks(n);
  hipLaunchKernelGGL(flux_pdf_kernel, dim3((unsigned)blocks), dim3(kPdfThreads), 0, st, F, n,
                     part);
  hipLaunchKernelGGL(flux_pdf_sum_kernel, dim3(kPdfSlots), dim3(64), 0, st, part, blocks, counts);
  return hipGetLastError();
}

hipError_t launch_twiddles(double2 *T, hipStream_t st) {
  hipLaunchKernelGGL(twiddle_kernel, dim3((kTwMax / 2 + 255) / 256), dim3(256), 0, st, T);
  return hipGetLastError();
}

hipError_t launch_flux_power(int64_t n_skewers, int max_n, const float *F, const int64_t *offsets,
                             const int64_t *mode_off, const float *dv, double inv_mean,
                             const double2 *T, float *P, uint32_t *status, hipStream_t st) {
  if (n_skewers <= 0) return hipSuccess;
  const int M = max_n / 2;
  const size_t lds = sizeof(double2) * (size_t)M;
  static bool attr_set[64] = {false};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev >= 0 && dev < 64 && !attr_set[dev]) {
    e = hipFuncSetAttribute((const void *)flux_power_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double2) * (kPsMaxN / 2 + kPsMaxN / 4)));
    if (e != hipSuccess) return e;
    attr_set[dev] = true;
  }
  hipLaunchKernelGGL(flux_power_kernel, dim3((unsigned)n_skewers), dim3(kPsThreads), lds, st, F,
                     offsets, mode_off, dv, inv_mean, T, P, status);
  return hipGetLastError();
}

}  // namespace lyaf
