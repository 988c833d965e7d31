// lyaf_instrument.hip -- the instrument model applied to the transmitted flux
// (Greig, Bolton & Wyithe 2011, Section 3.1 for the high-resolution mock
// spectra, Section 3.2 for the BOSS-like ones, Section 4.2 for the SDSS-like
// ones): convolution with a Gaussian line-spread function, resampling onto
// coarser bins, additive noise.
//
//   Fc_i   = sum_m c_m F_{(i-m) mod N},  c_m = g(m dv) / Z,  g(d) = exp(-(d/b_L)^2),
//            b_L = FWHM / (2 sqrt(ln 2)), m over |m dv| <= k b_L (or the whole
//            box at minimal images), Z = sum_m g(m dv)
//   Fbin_k = average over bin k ([v0 + k dv_bin, v0 + (k+1) dv_bin), periodic)
//            of the piecewise-constant spectrum that takes the value Fc_i on
//            pixel i = [(i - 1/2) dv, (i + 1/2) dv)
//   Fobs_k = Fbin_k + sigma eps_k
//
// Kernel layout.  A work item is (skewer, c): the bins whose lower edge lies in
// pixels [c W, (c+1) W) from the first bin's edge, W = kInsWindow.  Their pixel
// span (at most W + dv_bin/dv + 2 <= kInsTile pixels) is convolved in one
// workgroup: the flux with its halo of M pixels on each side is staged in LDS
// as FP64 in 8 planes by index mod 8 (lane l reads element 8l + j from plane
// j, so the reads of a wave are consecutive), each lane owns 8 consecutive
// outputs and walks the taps 8 at a time with a sliding window of registers,
// accumulating in FP64 (on gfx950 an FP64 FMA issues at the rate of an
// unpacked FP32 one).  Taps come in blocks of kInsTapBlock, so any line-spread
// width fits the same LDS.  The convolved span then becomes an FP64 prefix sum
// in LDS, and each bin is the difference of that cumulative integral, linearly
// interpolated, at its two edges, divided by its width.
//
// The backward kernel is the transpose: each pixel gathers the gradients of
// the bins it overlaps (times overlap / bin width), and the same convolution
// runs over those values (the taps are even in m).
#include "lyaf_internal.h"

namespace lyaf {
namespace {

constexpr int kInsThreads = 256;
constexpr int kInsPerLane = 8;                            // outputs per lane
constexpr int kInsTile = kInsThreads * kInsPerLane;       // 2048 pixels
constexpr int kInsWindow = 1792;                          // bin lower edges per item
constexpr int kInsTapBlock = 256;                         // taps staged at once
constexpr int kInsPlane = (kInsTile + kInsTapBlock) / 8;  // 288 doubles per plane
static_assert(kInsMaxRatio + kInsWindow + 4 <= kInsTile, "bin span must fit the tile");
static_assert(kInsTapBlock % 8 == 0, "tap blocks are walked 8 at a time");

// Per-skewer geometry shared by both kernels.
struct InsSkewer {
  int64_t off, n, out_off, n_out;
  double dv;   // pixel width, km/s
  double q;    // bin width in pixels
  int M;       // taps m = -M .. M
  bool half_ends;  // the two extreme taps are the same image (whole even box)
  bool ok;
};

__device__ InsSkewer ins_skewer(const InsArgs &a, int64_t s) {
  InsSkewer k;
  k.off = a.offsets[s];
  k.n = a.offsets[s + 1] - k.off;
  k.out_off = a.out_offsets[s];
  k.n_out = a.out_offsets[s + 1] - k.out_off;
  k.dv = (double)a.dv[s];
  k.q = a.bin / k.dv;
  k.ok = k.dv > 0.0 && isfinite(k.dv) &&
         (k.n_out == 0 || (k.q <= (double)kInsMaxRatio &&
                           (double)k.n_out * a.bin <= (double)k.n * k.dv * (1.0 + 1e-9)));
  k.M = 0;
  k.half_ends = false;
  if (a.fwhm > 0.0) {
    const double bL = a.fwhm * kInvTwoSqrtLn2;
    const double reach = a.window_k * bL / k.dv;  // taps with |m dv| <= k b_L
    if (a.window_k > 0.0 && reach < 0.5 * (double)(k.n - 1)) {
      k.M = (int)floor(reach);
    } else {  // the whole box, every offset at its minimal image
      k.M = (int)(k.n / 2);
      k.half_ends = (k.n % 2) == 0;
    }
  }
  return k;
}

// Lower edge of bin k in pixel coordinates (pixel i is [i, i+1)).
__device__ inline double bin_edge(const InsArgs &a, const InsSkewer &k, int64_t bin) {
  return (a.v_start + (double)bin * a.bin) / k.dv + 0.5;
}

__device__ inline int64_t wrap_index(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// LDS of one workgroup.
struct InsShared {
  double s[8 * kInsPlane];  // staged values in 8 planes, later the prefix sums
  double h[kInsTapBlock];   // taps of the current block
  double red[kInsThreads / 64];
};

// Sum over the workgroup, in a fixed order.
__device__ double block_sum_d(double v, double *red) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kInsThreads / 64; ++w) t += red[w];
  return t;
}

// Convolution of a tile: acc[q] = sum_{u < T} h_u src(base + 8l + q + u) for the
// lane's outputs t = 8l + q < span, with h_u = g((M - u) dv) (unnormalised;
// the sum of the taps is returned).  src(x) yields the value at staged offset
// x (x = 0 .. span + T - 2).
template <class Src>
__device__ double convolve_tile(const InsArgs &a, const InsSkewer &k, int span, Src src,
                                double (&acc)[kInsPerLane], InsShared &sh) {
  const int T = 2 * k.M + 1;
  const int tid = threadIdx.x;
  const bool wave_active = (tid & ~63) * kInsPerLane < span;
  const double inv_bL = a.fwhm > 0.0 ? 1.0 / (a.fwhm * kInvTwoSqrtLn2) : 0.0;
  double z_part = 0.0;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q) acc[q] = 0.0;
  for (int u0 = 0; u0 < T; u0 += kInsTapBlock) {
    const int tb = min(kInsTapBlock, T - u0);  // real taps in this block
    const int tbp = (tb + 7) & ~7;             // walked taps (zero-padded)
    __syncthreads();  // the previous block's readers are done
    for (int u = tid; u < tbp; u += kInsThreads) {
      double g = 0.0;
      if (u < tb) {
        const int m = k.M - (u0 + u);
        if (a.fwhm > 0.0) {
          const double x = (double)m * k.dv * inv_bL;
          g = exp(-x * x);
          if (k.half_ends && (m == k.M || m == -k.M)) g *= 0.5;
        } else {
          g = 1.0;  // M = 0: the identity
        }
      }
      sh.h[u] = g;
      z_part += g;
    }
    const int need = span + tbp - 1;  // staged offsets read by outputs < span
    const int real = span + tb - 1;   // offsets carrying real taps
    for (int x = tid; x < need; x += kInsThreads)
      sh.s[(x & 7) * kInsPlane + (x >> 3)] = x < real ? src(u0 + x) : 0.0;
    __syncthreads();
    if (wave_active) {
      const double *p = sh.s + tid;
      double wl[8], wh[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) wl[j] = p[j * kInsPlane];
      for (int u = 0; u < tbp; u += 8) {
        const int b = (u >> 3) + 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) wh[j] = p[j * kInsPlane + b];
        double hh[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) hh[i] = sh.h[u + i];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int q = 0; q < kInsPerLane; ++q) {
            const double w = (q + i < 8) ? wl[q + i] : wh[q + i - 8];
            acc[q] = __builtin_fma(hh[i], w, acc[q]);
          }
#pragma unroll
        for (int j = 0; j < 8; ++j) wl[j] = wh[j];
      }
    }
  }
  return block_sum_d(z_part, sh.red);
}

__global__ __launch_bounds__(kInsThreads) void instrument_kernel(InsArgs a,
                                                                 const int2 *__restrict__ items) {
  __shared__ InsShared sh;
  const int2 item = items[blockIdx.x];
  const InsSkewer k = ins_skewer(a, item.x);
  if (!k.ok) {
    if (item.y == 0 && threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
    return;
  }
  // bins of this item: lower edges in [c W, (c+1) W) pixels from the first edge
  const auto first_bin = [&](int64_t c) -> int64_t {
    if (c == 0) return 0;
    if (c * kInsWindow >= k.n) return k.n_out;  // past the last item
    const double kb = ceil((double)(c * kInsWindow) / k.q);
    return kb >= (double)k.n_out ? k.n_out : (int64_t)kb;
  };
  const int64_t k_lo = first_bin(item.y), k_hi = first_bin(item.y + 1);
  if (k_lo >= k_hi) return;
  const double xa = bin_edge(a, k, k_lo), xb = bin_edge(a, k, k_hi);
  const int64_t p0 = (int64_t)floor(xa);
  const int span = (int)((int64_t)floor(xb) - p0 + 1);
  if (span > kInsTile) {  // excluded by the bin-width limit; never expected
    if (threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
    return;
  }
  const float *F = a.in + k.off;
  const int64_t n = k.n;
  const int64_t base = wrap_index(p0 - k.M, n);
  const auto src = [&](int x) -> double {
    int64_t i = base + x;
    if (i >= n) i -= n;
    if (i >= n) i %= n;
    return (double)F[i];
  };
  double acc[kInsPerLane];
  const double Z = convolve_tile(a, k, span, src, acc, sh);

  // prefix sums of the convolved span: sh.s[t] = sum_{t' < t} Fc[t']
  const double invZ = 1.0 / Z;
  // only outputs inside the span enter the sums (lanes past it hold garbage)
  const int t0 = threadIdx.x * kInsPerLane;
  double run = 0.0, loc[kInsPerLane];
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q) {
    if (t0 + q < span) run += acc[q] * invZ;
    loc[q] = run;
  }
  // exclusive scan of the lane totals over the workgroup
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double incl = run;
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  __syncthreads();  // every wave is done with the staged values
  if (lane == 63) sh.red[wv] = incl;
  __syncthreads();
  double excl = incl - run;
  for (int w = 0; w < wv; ++w) excl += sh.red[w];
  if (threadIdx.x == 0) sh.s[0] = 0.0;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q)
    if (t0 + q < span) sh.s[t0 + q + 1] = excl + loc[q];
  __syncthreads();

  // bins: difference of the interpolated cumulative integral at their edges
  const auto cum = [&](double e) -> double {
    const int i = min((int)e, span - 1);
    const double f = e - (double)i;
    return sh.s[i] + f * (sh.s[i + 1] - sh.s[i]);
  };
  for (int64_t kb = k_lo + threadIdx.x; kb < k_hi; kb += kInsThreads) {
    const double e0 = bin_edge(a, k, kb) - (double)p0;
    const double e1 = bin_edge(a, k, kb + 1) - (double)p0;
    double v = (cum(e1) - cum(e0)) / (e1 - e0);
    if (a.noise) v += a.sigma * (double)a.noise[k.out_off + kb];
    a.out[k.out_off + kb] = (float)v;
  }
}

__global__ __launch_bounds__(kInsThreads) void instrument_backward_kernel(
    InsArgs a, const int2 *__restrict__ items) {
  __shared__ InsShared sh;
  const int2 item = items[blockIdx.x];
  const InsSkewer k = ins_skewer(a, item.x);
  if (!k.ok) {
    if (item.y == 0 && threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
    return;
  }
  const int64_t p0 = (int64_t)item.y * kInsTile;
  const int span = (int)min<int64_t>(kInsTile, k.n - p0);
  float *gF = a.out + k.off;
  if (k.n_out == 0) {
    for (int t = threadIdx.x; t < span; t += kInsThreads) gF[p0 + t] = 0.0f;
    return;
  }
  const int64_t n = k.n;
  const double nd = (double)n;
  const double x_first = bin_edge(a, k, 0), x_last = bin_edge(a, k, k.n_out);
  const float *g = a.in + k.out_off;
  const int64_t base = wrap_index(p0 - k.M, n);
  // gradient reaching convolved pixel i (0 <= i < n) from the bins over it
  const auto src = [&](int x) -> double {
    int64_t i = base + x;
    if (i >= n) i -= n;
    if (i >= n) i %= n;
    double v = 0.0;
    // images y = i + L n of the pixel that meet [x_first, x_last)
    const double L_lo = ceil((x_first - (double)i - 1.0) / nd);
    const double L_hi = floor((x_last - (double)i) / nd);
    for (double L = L_lo; L <= L_hi; L += 1.0) {
      const double y = (double)i + L * nd;
      int64_t kb = (int64_t)floor((y - x_first) / k.q) - 1;
      if (kb < 0) kb = 0;
      for (; kb < k.n_out; ++kb) {
        const double e0 = bin_edge(a, k, kb);
        if (e0 >= y + 1.0) break;
        const double e1 = bin_edge(a, k, kb + 1);
        const double ov = fmin(y + 1.0, e1) - fmax(y, e0);
        if (ov > 0.0) v += ov * (double)g[kb] / (e1 - e0);
      }
    }
    return v;
  };
  double acc[kInsPerLane];
  const double Z = convolve_tile(a, k, span, src, acc, sh);
  const double invZ = 1.0 / Z;
  const int t0 = threadIdx.x * kInsPerLane;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q)
    if (t0 + q < span) gF[p0 + t0 + q] = (float)(acc[q] * invZ);
}

}  // namespace

int ins_items_per_skewer(int64_t n, int64_t n_out, bool backward) {
  if (n <= 0) return 0;
  if (backward) return (int)((n + kInsTile - 1) / kInsTile);
  if (n_out <= 0) return 0;
  return (int)((n + kInsWindow - 1) / kInsWindow);
}

hipError_t launch_instrument(const InsArgs &a, const int2 *items, int64_t n_items, bool backward,
                             hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (backward)
    hipLaunchKernelGGL(instrument_backward_kernel, dim3((unsigned)n_items), dim3(kInsThreads), 0,
                       st, a, items);
  else
    hipLaunchKernelGGL(instrument_kernel, dim3((unsigned)n_items), dim3(kInsThreads), 0, st, a,
                       items);
  return hipGetLastError();
}

}  // namespace lyaf
