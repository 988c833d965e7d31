// lyaf_power3d.hip -- the 3D flux power spectrum reconstructed from a set of
// parallel sight-lines (Greig, Bolton & Wyithe 2011, Section 6.2, eq. 7).
//
// S sight-lines of n pixels run along z through the columns (x_s, y_s) of an
// n^3 periodic grid of side L; the flux contrast delta_s(z) = F_s(z)/Fbar - 1
// of each sits in its column with weight w_s (1 in the paper), the rest of the
// box is empty.  With unnormalised transforms
//   G_s(mz)   = sum_z delta_s(z) e^{-2 pi i mz z / n},
//   W(mx, my) = sum_s w_s e^{-2 pi i (mx x_s + my y_s) / n},
//   D(m)      = sum_s w_s G_s(mz) e^{-2 pi i (mx x_s + my y_s) / n},
// eq. (7) reads
//   P_true(m) = P_box(m) - [P_1D(mz) + P_N] P_2D,w(mx, my),
//   P_box = L^3 n^-6 |D|^2,  P_1D = L n^-2 mean_s |G_s|^2,  P_2D,w = L^2 n^-4 |W|^2,
// and the half-spectrum's modes (mz = 0 .. n/2; weight 2 for 0 < mz < n/2,
// which stand for their conjugate partners too) are averaged in spherical
// shells b <= |m| < b + 1 of the fundamental wavenumber: per shell the mode
// count, the mean |k| = 2 pi |m| / L, and the means of P_true and P_box.
//
// The 3D grid is never stored.  Kernels (all FP64):
//   p3d_line_kernel  one workgroup per sight-line: G_s by a half-length
//                    complex transform in LDS and the unpacking of the two
//                    real halves (as the 1D flux power);
//   p3d_p1d_kernel   P_1D(mz), fixed-order sums over chunks of sight-lines,
//                    then over the chunks (p3d_p1d_sum_kernel);
//   p3d_w_kernel     one workgroup per mx: the rows' weight sums
//                    sum_{s in row y} w_s e^{-2 pi i mx x_s / n}, placed in
//                    their rows, transformed along y: P_2D,w(mx, .);
//   p3d_x_kernel     one workgroup per (row y in use, 64 consecutive mz):
//                    D1(mx, y, mz) = sum_{s in row y} w_s G_s(mz) e^{-2 pi i mx x_s / n}
//                    for every mx (a direct sum over the row's few sight-lines);
//   p3d_y_kernel     persistent workgroups over (mx, run of C mz) items: the
//                    rows of D1 placed in an LDS column per mz (zeros in rows
//                    without sight-lines; the next item's rows read into
//                    registers meanwhile), transformed along y, then every
//                    mode's weighted P_box and P_true added into LDS shell
//                    sums with FP64 atomics; each workgroup writes its shells
//                    once.  The shells' mode counts and sums of |m| depend on
//                    the grid alone: the same kernel computes them without
//                    data once per grid and shell count, and the workspace
//                    keeps them;
//   p3d_bin_kernel   the shells of every workgroup summed in a fixed order,
//                    then the means (p3d_geom_sum_kernel likewise for the
//                    counts).
// Only the LDS atomics make the shell sums' order vary from run to run (the
// results agree to rounding, not bitwise).
#include <algorithm>

#include "lyaf_fft.h"
#include "lyaf_internal.h"

namespace lyaf {
namespace {

constexpr int kLineThreads = 256;
constexpr int kXThreads = 256;   // 4 waves: one mz per lane, waves split mx
constexpr int kXLines = 8;       // a row's sight-lines held in registers at once
constexpr int kYThreads = 1024;
constexpr int kYCap = 8192;      // n C complex doubles in LDS (128 KB)
constexpr int kBinThreads = 256;
constexpr int kP1dChunk = kP3dP1dChunk;

// e^{-2 pi i t / n} for 0 <= t < n from the half-period table.
__device__ inline double2 root_fwd(const double2 *__restrict__ T, int t, int n) {
  const int u = t * (kFftTableLen / n);
  return (u < kFftTableLen / 2) ? T[u]
                                : make_double2(-T[u - kFftTableLen / 2].x,
                                               -T[u - kFftTableLen / 2].y);
}

// G_s(mz), mz = 0 .. n/2, of delta_s = F_s / Fbar - 1: the n reals packed as
// M = n/2 complex values z_j = delta_{2j} + i delta_{2j+1}, transformed, then
// X_m = E_m + e^{-pi i m / M} O_m, E_m = (Z_m + conj Z_{M-m}) / 2,
// O_m = (Z_m - conj Z_{M-m}) / 2i.
__global__ __launch_bounds__(kLineThreads) void p3d_line_kernel(P3dArgs a) {
  extern __shared__ double2 lds_line[];  // [n/2]
  const int s = blockIdx.x;
  const int n = a.n, M = n / 2;
  const float *f = a.F + (size_t)s * n;
  for (int j = threadIdx.x; j < M; j += kLineThreads)
    lds_line[j] = make_double2(__builtin_fma((double)f[2 * j], a.inv_mean, -1.0),
                               __builtin_fma((double)f[2 * j + 1], a.inv_mean, -1.0));
  __syncthreads();
  fft_batch<kLineThreads, kP3dMaxN / 2>(lds_line, a.twiddle, M, 0);
  double s1, c1;
  sincospi(-1.0 / (double)M, &s1, &c1);
  const double2 half_step = make_double2(c1, s1);
  double2 *out = a.G + (size_t)s * a.H;
  for (int m = threadIdx.x; m <= M; m += kLineThreads) {
    const double2 zm = lds_line[m == M ? 0 : m];
    const double2 zc = conj(lds_line[m == 0 ? 0 : M - m]);
    const double2 E = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
    const double2 d = csub(zm, zc);
    const double2 O = make_double2(0.5 * d.y, -0.5 * d.x);
    double2 tw;
    if (m == M) {
      tw = make_double2(-1.0, 0.0);
    } else {
      tw = a.twiddle[(m >> 1) * (kFftTableLen / M)];  // e^{-2 pi i (m >> 1) / M}
      if (m & 1) tw = cmul(tw, half_step);
    }
    out[m] = cadd(E, cmul(tw, O));
  }
}

// P_1D(mz) = L n^-2 (1/S) sum_s |G_s(mz)|^2 in two fixed-order stages:
// workgroup (mz block of 64, chunk of kP1dChunk sight-lines) sums its chunk
// (each wave a strided quarter of it, then the four waves in order) into
// part[chunk][mz]; p3d_p1d_sum_kernel adds the chunks in order.
__global__ __launch_bounds__(256) void p3d_p1d_kernel(P3dArgs a, int n_kzb) {
  __shared__ double sh[256];
  const int kzb = (int)blockIdx.x % n_kzb, chunk = (int)blockIdx.x / n_kzb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kz = kzb * 64 + lane;
  const int s_end = min(a.n_lines, (chunk + 1) * kP1dChunk);
  double acc = 0.0;
  if (kz < a.H)
    for (int s = chunk * kP1dChunk + wave; s < s_end; s += 4) {
      const double2 g = a.G[(size_t)s * a.H + kz];
      acc = __builtin_fma(g.x, g.x, __builtin_fma(g.y, g.y, acc));
    }
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (wave == 0 && kz < a.H)
    a.p1d_part[(size_t)chunk * a.H + kz] = ((sh[lane] + sh[64 + lane]) + sh[128 + lane]) +
                                           sh[192 + lane];
}

__global__ __launch_bounds__(256) void p3d_p1d_sum_kernel(P3dArgs a, int n_chunks) {
  const int kz = blockIdx.x * 256 + threadIdx.x;
  if (kz >= a.H) return;
  double acc = 0.0;
  for (int c = 0; c < n_chunks; ++c) acc += a.p1d_part[(size_t)c * a.H + kz];
  const double n = (double)a.n;
  a.P1d[kz] = a.L / (n * n) * acc / (double)a.n_lines;
}

// P_2D,w(mx, my) for one mx: the rows' weight sums placed in their rows, one
// forward transform along y.
__global__ __launch_bounds__(kLineThreads) void p3d_w_kernel(P3dArgs a) {
  extern __shared__ double2 lds_w[];  // [n]
  const int kx = blockIdx.x;
  const int n = a.n;
  for (int y = threadIdx.x; y < n; y += kLineThreads) lds_w[y] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int r = threadIdx.x; r < a.n_rows; r += kLineThreads) {
    double2 acc = make_double2(0.0, 0.0);
    for (int i = a.row_first[r]; i < a.row_first[r + 1]; ++i) {
      const int2 l = a.lines[i];
      const double wt = a.w ? a.w[l.x] : 1.0;
      const double2 e = root_fwd(a.twiddle, (int)(((int64_t)kx * l.y) & (n - 1)), n);
      acc.x = __builtin_fma(wt, e.x, acc.x);
      acc.y = __builtin_fma(wt, e.y, acc.y);
    }
    lds_w[a.rows[r]] = acc;
  }
  __syncthreads();
  fft_batch<kLineThreads, kP3dMaxN>(lds_w, a.twiddle, n, 0);
  const double nn = (double)n * (double)n;
  const double scale = a.L * a.L / (nn * nn);
  for (int y = threadIdx.x; y < n; y += kLineThreads) {
    const double2 v = lds_w[y];
    a.P2d[(size_t)kx * n + y] = scale * __builtin_fma(v.x, v.x, v.y * v.y);
  }
}

// D1(mx, y_r, mz) for every mx, one row r and 64 consecutive mz.
__global__ __launch_bounds__(kXThreads) void p3d_x_kernel(P3dArgs a, int n_kzb) {
  __shared__ double2 tw[kP3dMaxN];
  const int r = (int)blockIdx.x / n_kzb;
  const int kzb = (int)blockIdx.x - r * n_kzb;
  const int n = a.n, H = a.H;
  for (int t = threadIdx.x; t < n; t += kXThreads) tw[t] = root_fwd(a.twiddle, t, n);
  const int first = a.row_first[r], cnt = a.row_first[r + 1] - first;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kz = kzb * 64 + lane;
  const bool valid = kz < H;
  // the row's first kXLines sight-lines, weighted, in registers
  double2 g[kXLines];
  int xs[kXLines];
#pragma unroll
  for (int m = 0; m < kXLines; ++m) {
    xs[m] = 0;
    g[m] = make_double2(0.0, 0.0);
    if (m < cnt) {
      const int2 l = a.lines[first + m];
      xs[m] = l.y;
      const double wt = a.w ? a.w[l.x] : 1.0;
      const double2 v = valid ? a.G[(size_t)l.x * H + kz] : make_double2(0.0, 0.0);
      g[m] = make_double2(wt * v.x, wt * v.y);
    }
  }
  __syncthreads();
  const int mask = n - 1;
  for (int kx = wave; kx < n; kx += kXThreads / 64) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int m = 0; m < kXLines; ++m) {
      if (m < cnt) {
        const double2 e = tw[(kx * xs[m]) & mask];
        acc.x = __builtin_fma(g[m].x, e.x, __builtin_fma(-g[m].y, e.y, acc.x));
        acc.y = __builtin_fma(g[m].x, e.y, __builtin_fma(g[m].y, e.x, acc.y));
      }
    }
    for (int m = kXLines; m < cnt; ++m) {  // crowded rows: the rest from memory
      const int2 l = a.lines[first + m];
      const double wt = a.w ? a.w[l.x] : 1.0;
      const double2 v = valid ? a.G[(size_t)l.x * H + kz] : make_double2(0.0, 0.0);
      const double2 e = tw[(kx * l.y) & mask];
      const double gx = wt * v.x, gy = wt * v.y;
      acc.x = __builtin_fma(gx, e.x, __builtin_fma(-gy, e.y, acc.x));
      acc.y = __builtin_fma(gx, e.y, __builtin_fma(gy, e.x, acc.y));
    }
    if (valid) a.D1[((size_t)kx * a.n_rows + r) * H + kz] = acc;
  }
}

// Shell index and weight of mode (mx, my, mz) on the half-spectrum.
__device__ inline int shell_of(int mx, int my, int mz, int n, double &m, double &wt) {
  m = sqrt((double)(mx * mx + my * my + mz * mz));
  wt = (mz == 0 || mz == n / 2) ? 1.0 : 2.0;
  return (int)m;  // floor: m >= 0
}

// The transform along y of (mx, run of C mz) items, and the shell sums of
// P_true and P_box.  Each workgroup loops over items with the next item's rows
// of D1 read into registers while the current one is transformed and binned
// (the transform's barriers wait for LDS traffic only); every mode adds its two
// weighted powers into LDS shell sums with FP64 atomics, and each workgroup
// writes its shells once.  GEOM = true runs the same loop over the modes
// without data: the shells' mode counts and sums of weighted |m|, which depend
// only on the grid and are kept by the caller across calls.
template <bool GEOM>
__global__ __launch_bounds__(kYThreads) void p3d_y_kernel(P3dArgs a, int lgC, int n_chunks,
                                                          int nb) {
  extern __shared__ double2 lds_y[];  // [n][C], then 2 nb shell sums
  const int n = a.n, H = a.H, C = 1 << lgC;
  double *bins = reinterpret_cast<double *>(lds_y + (GEOM ? 0 : (n << lgC)));
  for (int i = threadIdx.x; i < 2 * nb; i += kYThreads) bins[i] = 0.0;
  const double nn = (double)n * (double)n;
  const double box_scale = a.L * a.L * a.L / (nn * nn * nn);
  const int n_items = n * n_chunks;
  const int n_el = n << lgC;
  constexpr int E = kYCap / kYThreads;  // elements per thread
  double2 nxt[E];
  // element q = threadIdx.x + e kYThreads is (y = q >> lgC, column c = q & (C-1))
  auto fetch = [&](int item) {
    const int kx = item / n_chunks;
    const int kz0 = (item - kx * n_chunks) * C;
    const double2 *src = a.D1 + (size_t)kx * a.n_rows * H + kz0;
    int tx = (int)threadIdx.x;
    asm volatile("" : "+v"(tx));  // indices per item, not hoisted out of the loop
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = tx + e * kYThreads;
      nxt[e] = make_double2(0.0, 0.0);
      if (q < n_el) {
        const int r = a.row_of_y[q >> lgC], c = q & (C - 1);
        if (r >= 0 && kz0 + c < H) nxt[e] = src[(size_t)r * H + c];
      }
    }
  };
  int item = blockIdx.x;
  if (!GEOM && item < n_items) fetch(item);
  __syncthreads();  // the shell sums are cleared
  for (; item < n_items; item += gridDim.x) {
    const int kx = item / n_chunks;
    const int kz0 = (item - kx * n_chunks) * C;
    const int mx = kx <= n / 2 ? kx : kx - n;
    if (!GEOM) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int q = (int)threadIdx.x + e * kYThreads;
        if (q < n_el) lds_y[q] = nxt[e];
      }
      lds_barrier();
      if (item + (int)gridDim.x < n_items) fetch(item + gridDim.x);  // in flight meanwhile
      fft_batch<kYThreads, kYCap>(lds_y, a.twiddle, n, lgC);
    }
    for (int q = threadIdx.x; q < n_el; q += kYThreads) {
      const int ky = q >> lgC, c = q & (C - 1);
      const int kz = kz0 + c;
      if (kz >= H) continue;
      const int my = ky <= n / 2 ? ky : ky - n;
      double m, wt;
      const int b = shell_of(mx, my, kz, n, m, wt);
      if (b >= nb) continue;
      if (GEOM) {
        atomicAdd(&bins[b], wt);
        atomicAdd(&bins[nb + b], wt * m);
      } else {
        const double2 D = lds_y[q];
        const double pbox = box_scale * __builtin_fma(D.x, D.x, D.y * D.y);
        const double ptrue = pbox - (a.P1d[kz] + a.p_noise) * a.P2d[(size_t)kx * n + ky];
        atomicAdd(&bins[b], wt * ptrue);
        atomicAdd(&bins[nb + b], wt * pbox);
      }
    }
    if (!GEOM) lds_barrier();  // the next item overwrites the buffer
  }
  __syncthreads();
  double *out = (GEOM ? a.geom_part : a.shells) + (size_t)blockIdx.x * 2 * nb;
  for (int i = threadIdx.x; i < 2 * nb; i += kYThreads) out[i] = bins[i];
}

// The shells' mode counts and sums of weighted |m|, summed over the
// workgroups of the geometry pass in a fixed order.
__global__ __launch_bounds__(kBinThreads) void p3d_geom_sum_kernel(P3dArgs a, int nb,
                                                                   int n_parts) {
  const int b = blockIdx.x * kBinThreads + threadIdx.x;
  if (b >= nb) return;
  double t0 = 0.0, t1 = 0.0;
  for (int p = 0; p < n_parts; ++p) {
    const double *s = a.geom_part + (size_t)p * 2 * nb;
    t0 += s[b];
    t1 += s[nb + b];
  }
  a.geom[b] = t0;
  a.geom[nb + b] = t1;
}

// Sum the workgroups' shells in a fixed order; means per shell.
__global__ __launch_bounds__(kBinThreads) void p3d_bin_kernel(P3dArgs a, int nb, int n_parts) {
  const int b = blockIdx.x * kBinThreads + threadIdx.x;
  if (b >= a.n_bins) return;
  double cnt = 0.0, km = 0.0, pt = 0.0, pb = 0.0;
  if (b < nb) {
    cnt = a.geom[b];
    km = a.geom[nb + b];
    for (int p = 0; p < n_parts; ++p) {
      const double *s = a.shells + (size_t)p * 2 * nb;
      pt += s[b];
      pb += s[nb + b];
    }
  }
  const bool any = cnt > 0.0;
  a.counts[b] = cnt;
  a.k_mean[b] = any ? km / cnt * (2.0 * M_PI / a.L) : 0.0;
  a.p_true[b] = any ? pt / cnt : 0.0;
  a.p_box[b] = any ? pb / cnt : 0.0;
}

bool g_attr_set[64] = {false};
int g_resident[64] = {0};

}  // namespace

int p3d_shell_bins(int n, int n_bins) {
  // largest |m| on the half-spectrum: sqrt(3) n / 2
  const int bmax = (int)floor(sqrt(3.0) * n / 2.0);
  return std::min(n_bins, bmax + 1);
}

// mz columns per p3d_y item: the largest power of two (at most 16) whose
// n C complex doubles fit kYCap and, with the shell sums of the largest
// shell count, the LDS of one workgroup.
int p3d_y_columns(int n) {
  const size_t bins = 2 * sizeof(double) * (size_t)p3d_shell_bins(n, INT32_MAX);
  int C = 16;
  while (C > 1 && ((size_t)n * C > (size_t)kYCap ||
                   sizeof(double2) * (size_t)n * C + bins > (size_t)kP3dMaxLds))
    C >>= 1;
  return C;
}

hipError_t p3d_kernel_attributes(int n, int nb, int *y_grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!g_attr_set[dev]) {
    if ((e = hipFuncSetAttribute((const void *)p3d_y_kernel<false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kP3dMaxLds)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)p3d_y_kernel<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kP3dMaxLds)) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute((const void *)p3d_w_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(sizeof(double2) * kP3dMaxN))) != hipSuccess)
      return e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return e;
    g_resident[dev] = prop.multiProcessorCount;
    g_attr_set[dev] = true;
  }
  const int C = p3d_y_columns(n);
  const size_t lds = sizeof(double2) * (size_t)n * C + 2 * sizeof(double) * (size_t)nb;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)p3d_y_kernel<false>,
                                                        kYThreads, lds)) != hipSuccess)
    return e;
  *y_grid = std::max(1, per_cu) * g_resident[dev];
  return hipSuccess;
}

hipError_t launch_power3d(const P3dArgs &a, int y_grid, bool need_geom, hipStream_t st) {
  const int n = a.n;
  const int C = p3d_y_columns(n);
  int lgC = 0;
  while ((1 << lgC) < C) ++lgC;
  const int n_chunks = (a.H + C - 1) / C;
  const int nb = p3d_shell_bins(n, a.n_bins);
  const int grid = std::min(y_grid, n * n_chunks);
  if (need_geom) {  // once per grid and shell count: counts and mean |k|
    hipLaunchKernelGGL(p3d_y_kernel<true>, dim3(grid), dim3(kYThreads),
                       2 * sizeof(double) * (size_t)nb, st, a, lgC, n_chunks, nb);
    hipLaunchKernelGGL(p3d_geom_sum_kernel, dim3((nb + kBinThreads - 1) / kBinThreads),
                       dim3(kBinThreads), 0, st, a, nb, grid);
  }
  hipLaunchKernelGGL(p3d_line_kernel, dim3(a.n_lines), dim3(kLineThreads),
                     sizeof(double2) * (size_t)(n / 2), st, a);
  const int p1d_kzb = (a.H + 63) / 64;
  const int p1d_chunks = (a.n_lines + kP1dChunk - 1) / kP1dChunk;
  hipLaunchKernelGGL(p3d_p1d_kernel, dim3(p1d_kzb * p1d_chunks), dim3(256), 0, st, a, p1d_kzb);
  hipLaunchKernelGGL(p3d_p1d_sum_kernel, dim3((a.H + 255) / 256), dim3(256), 0, st, a,
                     p1d_chunks);
  hipLaunchKernelGGL(p3d_w_kernel, dim3(n), dim3(kLineThreads), sizeof(double2) * (size_t)n,
                     st, a);
  const int n_kzb = (a.H + 63) / 64;
  hipLaunchKernelGGL(p3d_x_kernel, dim3(a.n_rows * n_kzb), dim3(kXThreads), 0, st, a, n_kzb);
  hipLaunchKernelGGL(p3d_y_kernel<false>, dim3(grid), dim3(kYThreads),
                     sizeof(double2) * (size_t)(n << lgC) + 2 * sizeof(double) * (size_t)nb,
                     st, a, lgC, n_chunks, nb);
  hipLaunchKernelGGL(p3d_bin_kernel, dim3((a.n_bins + kBinThreads - 1) / kBinThreads),
                     dim3(kBinThreads), 0, st, a, nb, grid);
  return hipGetLastError();
}

}  // namespace lyaf
