// lyaf_fields.hip -- skewer-only synthesis of the linear density and velocity
// fields (Greig, Bolton & Wyithe 2011, Section 2.1 and Appendix B).
//
// A Gaussian field g(k) is given on the half-spectrum of a real N^3 grid of a
// periodic box of side L (k = 2 pi (mx, my, mz) / L, mx and my signed, mz = 0 ..
// N/2).  The dark-matter field is delta_DM = amp sqrt(P(|k|)) g, with P
// linearly interpolated from a table; the baryons follow the filter of eq. (1),
// delta_b = delta_DM / (1 + k^2 / k_F^2); the velocity follows eq. (3),
// v = E_+ i k / k^2 delta_DM, of which the component along the sight-lines (z)
// is kept.  Only the S requested sight-lines (columns (x_s, y_s)) are brought
// back to real space, as Appendix B does it: transforms across the (kx, ky)
// planes, then one 1D transform per sight-line.  For each field F:
//
//   f_s(z) = N^-3 sum_mz c_mz Re[ C_s(mz) e^{2 pi i mz z / N} ],  c = 1 at mz = 0, N/2, else 2,
//   C_s(mz) = sum_mx e^{2 pi i mx x_s / N} T(mx, y_s, mz),
//   T(mx, y, mz) = sum_my e^{2 pi i my y / N} F(mx, my, mz).
//
// Three kernels, all reading their inputs once:
//   field_ky_kernel  persistent workgroups over (mx, run of C consecutive mz)
//                    items, the next item's modes read ahead: reads the
//                    N x C modes (C consecutive mz are contiguous), forms both
//                    fields' spectra (FP32 multipliers), inverse-transforms
//                    the 2C columns along my in LDS as one batch (FP32,
//                    Stockham passes) and
//                    writes only the rows y that some sight-line uses:
//                    T [rows][N][N/2+1] complex float per field;
//   field_kx_kernel  one workgroup per (group of up to 8 sight-lines sharing a
//                    row y, 256 consecutive mz): each thread owns one mz and
//                    sums over mx for every sight-line of the group, in FP64,
//                    twiddles from an LDS table: C [S][N/2+1] complex double;
//   field_z_kernel   one workgroup per sight-line: both real fields as the real
//                    and imaginary parts of one complex inverse transform
//                    (Hermitian extension of each half-spectrum), FP64 in LDS,
//                    scaled by N^-3 and stored as float.
#include <algorithm>

#include "lyaf_fft.h"
#include "lyaf_internal.h"

namespace lyaf {
namespace {

constexpr int kKyThreads = 1024;
constexpr int kKyCap = 16384;  // N 2C complex floats in LDS (128 KB)
constexpr int kKxThreads = 256;
constexpr int kKxLines = kFieldLinesPerGroup;  // sight-lines per group
constexpr int kZThreads = 256;

// Multiplier of g for each field at integer wavenumber (mx, my, mz): the
// baryon field's real factor and the velocity's real factor (times i).
__device__ inline void field_factors(const FieldArgs &a, int mx, int my, int mz, float &fb,
                                     float &fv) {
  const int m2 = mx * mx + my * my + mz * mz;  // exact: at most 3 (N/2)^2
  const float m2f = (float)m2;
  const float kmag = a.kfun * __builtin_sqrtf(m2f);
  const float x = kmag * a.inv_dk;
  const int j = (int)x;  // x >= 0
  float P = 0.f;
  if (j + 1 < a.n_table) {
    const float p0 = (float)a.pk[j], p1 = (float)a.pk[j + 1];
    P = __builtin_fmaf(x - (float)j, p1 - p0, p0);
  } else if (j + 1 == a.n_table && x == (float)j) {
    P = (float)a.pk[j];  // exactly at the last node
  }
  const float A = a.amp * __builtin_sqrtf(fmaxf(P, 0.f));
  fb = A / __builtin_fmaf(a.kfun2_inv_kF2, m2f, 1.f);
  fv = (m2 > 0) ? a.E_over_kfun * (float)mz / m2f * A : 0.f;
}

// Block index -> work item with the items of each XCD contiguous: workgroup b
// runs on XCD b mod 8, so neighbouring mz runs of one mx (which share cache
// lines) are taken by the same L2.
__device__ inline int xcd_item(int n_items) {
  const int per = (int)gridDim.x >> 3;  // gridDim.x is a multiple of 8
  const int b = (int)blockIdx.x;
  const int item = (b & 7) * per + (b >> 3);
  return item < n_items ? item : -1;
}

// Persistent: workgroup b takes items b', b' + G, .. (G workgroups; b' puts
// the workgroups of one XCD on consecutive items, whose mz runs share cache
// lines), and reads the next item's modes into registers while the current
// one is transformed and stored.
__global__ __launch_bounds__(kKyThreads) void field_ky_kernel(FieldArgs a, int lgC,
                                                               int n_chunks) {
  // [N][2][C]: both fields' C columns side by side, one batch of 2C transforms
  extern __shared__ float2 lds_ky[];
  const int N = a.N, H = a.H;
  const int C = 1 << lgC;
  const int n_items = N * n_chunks;
  const int n_el = N << lgC;
  const int G = (int)gridDim.x;  // a multiple of 8
  const int first = ((int)blockIdx.x & 7) * (G >> 3) + ((int)blockIdx.x >> 3);
  constexpr int E = kKyCap / 2 / kKyThreads;  // modes per thread per item
  float2 nxt[E];
  auto fetch = [&](int item) {
    const int kx = item / n_chunks;
    const int kz0 = (item - kx * n_chunks) * C;
    const float2 *src = a.modes + (size_t)kx * N * H + kz0;
    int tx = (int)threadIdx.x;
    asm volatile("" : "+v"(tx));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = tx + e * kKyThreads;
      nxt[e] = make_float2(0.f, 0.f);
      if (q < n_el && kz0 + (q & (C - 1)) < H) nxt[e] = src[(size_t)(q >> lgC) * H + (q & (C - 1))];
    }
  };
  if (first < n_items) fetch(first);
  for (int item = first; item < n_items; item += G) {
    const int kx = item / n_chunks;
    const int kz0 = (item - kx * n_chunks) * C;
    const int mx = kx <= N / 2 ? kx : kx - N;
    // the per-element indices below are recomputed for every item: hoisted out
    // of the item loop they would hold E sets of registers for its whole length
    int tx = (int)threadIdx.x;
    asm volatile("" : "+v"(tx));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = tx + e * kKyThreads;
      if (q < n_el) {
        const int ky = q >> lgC, c = q & (C - 1);
        float2 b = make_float2(0.f, 0.f), v = make_float2(0.f, 0.f);
        if (kz0 + c < H) {
          const float2 g = nxt[e];
          float fb, fv;
          field_factors(a, mx, ky <= N / 2 ? ky : ky - N, kz0 + c, fb, fv);
          // conjugated on the way in: the inverse transform is conj(FFT(conj))
          b = make_float2(g.x * fb, -g.y * fb);
          v = make_float2(-g.y * fv, -g.x * fv);  // conj(i fv g)
        }
        lds_ky[(ky << (lgC + 1)) + c] = b;
        lds_ky[(ky << (lgC + 1)) + C + c] = v;
      }
      asm volatile("" ::: "memory");  // one element's multipliers at a time
    }
    lds_barrier();
    if (item + G < n_items) fetch(item + G);  // in flight during the transform
    fft_batch<kKyThreads, kKyCap>(lds_ky, a.twiddle, N, lgC + 1);
    const int n_out = a.n_rows << (lgC + 1);
    for (int q = threadIdx.x; q < n_out; q += kKyThreads) {
      const int yi = q >> (lgC + 1), f = (q >> lgC) & 1, c = q & (C - 1);
      if (kz0 + c < H) {
        float2 *dst = (f == 0 ? a.Tb : a.Tv) + ((size_t)yi * N + kx) * H + kz0 + c;
        *dst = conj(lds_ky[(a.rows[yi] << (lgC + 1)) + (f << lgC) + c]);
      }
    }
    lds_barrier();  // every read of the buffer is done before the next item
  }
}

// e^{+2 pi i t / N} for t < N from the half-period table of e^{-2 pi i u / 4096}.
__device__ inline double2 root_of_unity(const double2 *__restrict__ T, int t, int N) {
  const int u = t * (kFftTableLen / N);
  const double2 w = (u < kFftTableLen / 2) ? T[u] : make_double2(-T[u - kFftTableLen / 2].x,
                                                                  -T[u - kFftTableLen / 2].y);
  return conj(w);
}

__global__ __launch_bounds__(kKxThreads) void field_kx_kernel(FieldArgs a, int n_kzb) {
  extern __shared__ double2 tw[];  // [N]
  const int g = (int)blockIdx.x / n_kzb;
  const int kzb = (int)blockIdx.x - g * n_kzb;
  const int N = a.N, H = a.H;
  const int4 grp = a.groups[g];  // (row, first line, count, -)
  for (int t = threadIdx.x; t < N; t += kKxThreads) tw[t] = root_of_unity(a.twiddle, t, N);
  int xs[kKxLines];
#pragma unroll
  for (int m = 0; m < kKxLines; ++m) xs[m] = m < grp.z ? a.lines[grp.y + m].y : 0;
  __syncthreads();
  const int kz = kzb * kKxThreads + (int)threadIdx.x;
  if (kz - (int)(threadIdx.x & 63) >= H) return;  // the wave holds no mz
  const bool valid = kz < H;
  const size_t base = (size_t)grp.x * N * H + (valid ? kz : 0);
  const float2 *rb = a.Tb + base;
  const float2 *rv = a.Tv + base;
  double2 ab[kKxLines], av[kKxLines];
#pragma unroll
  for (int m = 0; m < kKxLines; ++m) {
    ab[m] = make_double2(0.0, 0.0);
    av[m] = make_double2(0.0, 0.0);
  }
  int idx[kKxLines];  // (kx x_m) mod N
#pragma unroll
  for (int m = 0; m < kKxLines; ++m) idx[m] = 0;
  const int mask = N - 1;
  constexpr int U = 4;  // rows of T in flight per thread
  for (int kx0 = 0; kx0 < N; kx0 += U) {
    float2 tb[U], tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = valid && kx0 + u < N;
      tb[u] = in ? rb[(size_t)(kx0 + u) * H] : make_float2(0.f, 0.f);
      tv[u] = in ? rv[(size_t)(kx0 + u) * H] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double bx = tb[u].x, by = tb[u].y, vx = tv[u].x, vy = tv[u].y;
#pragma unroll
      for (int m = 0; m < kKxLines; ++m) {
        if (m < grp.z) {
          const double2 w = tw[idx[m]];
          ab[m].x = __builtin_fma(bx, w.x, __builtin_fma(-by, w.y, ab[m].x));
          ab[m].y = __builtin_fma(bx, w.y, __builtin_fma(by, w.x, ab[m].y));
          av[m].x = __builtin_fma(vx, w.x, __builtin_fma(-vy, w.y, av[m].x));
          av[m].y = __builtin_fma(vx, w.y, __builtin_fma(vy, w.x, av[m].y));
          idx[m] = (idx[m] + xs[m]) & mask;
        }
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int m = 0; m < kKxLines; ++m) {
    if (m < grp.z) {
      const size_t s = (size_t)a.lines[grp.y + m].x;
      a.Cb[s * H + kz] = ab[m];
      a.Cv[s * H + kz] = av[m];
    }
  }
}

__global__ __launch_bounds__(kZThreads) void field_z_kernel(FieldArgs a) {
  extern __shared__ double2 lds_z[];  // [N]
  const int s = blockIdx.x;
  const int N = a.N, H = a.H, half = N / 2;
  const double2 *cb = a.Cb + (size_t)s * H;
  const double2 *cv = a.Cv + (size_t)s * H;
  for (int k = threadIdx.x; k < N; k += kZThreads) {
    double2 z;
    if (k == 0 || k == half) {
      z = make_double2(cb[k].x, cv[k].x);  // the imaginary parts drop out of Re[]
    } else if (k < half) {
      const double2 b = cb[k], v = cv[k];
      z = make_double2(b.x - v.y, b.y + v.x);  // C_b + i C_v
    } else {
      const double2 b = cb[N - k], v = cv[N - k];
      z = make_double2(b.x + v.y, v.x - b.y);  // conj(C_b) + i conj(C_v)
    }
    lds_z[k] = conj(z);
  }
  __syncthreads();
  fft_batch<kZThreads, kFieldMaxN>(lds_z, a.twiddle, N, 0);
  const double scale = a.inv_n3;
  float *ob = a.delta_b + (size_t)s * N;
  float *ov = a.v_z + (size_t)s * N;
  for (int t = threadIdx.x; t < N; t += kZThreads) {
    const double2 z = lds_z[t];  // conj of the inverse transform: f_b - i f_v
    ob[t] = (float)(z.x * scale);
    ov[t] = (float)(-z.y * scale);
  }
}

bool g_attr_set[64] = {false};

}  // namespace

int field_ky_columns(int N) { return std::min(16, kKyCap / (2 * N)); }

int g_ky_resident[64] = {0};

hipError_t field_kernel_attributes(int *ky_resident) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (g_attr_set[dev]) {
    *ky_resident = g_ky_resident[dev];
    return hipSuccess;
  }
  if ((e = hipFuncSetAttribute((const void *)field_ky_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(float2) * kKyCap))) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void *)field_z_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(double2) * kFieldMaxN))) != hipSuccess)
    return e;
  int per_cu = 0, cus = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)field_ky_kernel,
                                                        kKyThreads,
                                                        sizeof(float2) * kKyCap)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
          hipSuccess)
    return e;
  g_ky_resident[dev] = std::max(1, per_cu) * cus;
  g_attr_set[dev] = true;
  *ky_resident = g_ky_resident[dev];
  return hipSuccess;
}

hipError_t launch_field_ky(const FieldArgs &a, int resident, hipStream_t st) {
  const int C = field_ky_columns(a.N);
  int lgC = 0;
  while ((1 << lgC) < C) ++lgC;
  const int n_chunks = (a.H + C - 1) / C;
  const int items = a.N * n_chunks;
  // persistent: the resident workgroups, at most the items, a multiple of 8
  const int grid = std::max(8, std::min(resident, (items + 7) / 8 * 8) / 8 * 8);
  hipLaunchKernelGGL(field_ky_kernel, dim3(grid), dim3(kKyThreads),
                     sizeof(float2) * (size_t)(a.N << (lgC + 1)), st, a, lgC, n_chunks);
  return hipGetLastError();
}

hipError_t launch_field_kx(const FieldArgs &a, int n_groups, hipStream_t st) {
  const int n_kzb = (a.H + kKxThreads - 1) / kKxThreads;
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(field_kx_kernel, dim3(n_groups * n_kzb), dim3(kKxThreads),
                     sizeof(double2) * (size_t)a.N, st, a,
                     n_kzb);
  return hipGetLastError();
}

hipError_t launch_field_z(const FieldArgs &a, int n_lines, hipStream_t st) {
  if (n_lines <= 0) return hipSuccess;
  hipLaunchKernelGGL(field_z_kernel, dim3(n_lines), dim3(kZThreads),
                     sizeof(double2) * (size_t)a.N, st, a);
  return hipGetLastError();
}

}  // namespace lyaf
