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
// Kernel layout.  The forward takes one skewer per workgroup and walks its
// tiles: tile c holds the bins whose lower edge lies in pixels [c W, (c+1) W)
// from the first bin's edge, W = kInsWindow, and their pixel span (at most
// W + dv_bin/dv + 2 <= kInsTile pixels) is convolved by the workgroup.  The
// flux of a tile with its halo of M pixels on each side sits in LDS in 8 planes
// by index mod 8 (lane l reads element 8l + j from plane j, so the reads of a
// wave are consecutive); each lane owns 8 consecutive outputs and walks the
// taps 16 at a time with two windows of registers used in turn, accumulating
// in FP64 (on gfx950 an FP64 FMA issues at the rate of an unpacked FP32 one).
// When the taps fit one block of kInsTapBlock, the skewer's taps are formed
// once and the flux is staged as FP32 in two buffers: the next tile is copied
// from memory straight into the other buffer (global_load_lds, one wave
// instruction per plane and 64 rows) while this one is convolved.  Wider
// line-spread functions stage FP64 values and the taps block by block for every
// tile (the plane stride puts those 8 planes on different banks).  The
// convolved span then becomes an FP64 prefix sum in LDS, and each bin is the
// difference of that cumulative integral, linearly interpolated, at its two
// edges, divided by its width.
//
// The backward is the transpose: each pixel gathers the gradients of the bins
// it overlaps (times overlap / bin width), and the same convolution runs over
// those values (the taps are even in m).  Skewers with at most kInsBwdBins
// bins take one workgroup each, which forms the bins' FP64 prefix sums once in
// LDS (a pixel's gathered gradient is then the difference of their linear
// interpolation at its two edges) and walks the skewer's tiles, gathering a
// row of 8 staged pixels per thread and the few rows past one per thread a
// pixel per thread; skewers with more bins take one workgroup per tile and
// gather by a merge walk over the bins in memory.
#include <algorithm>

#include "lyaf_internal.h"

namespace lyaf {
namespace {

constexpr int kInsThreads = 256;
constexpr int kInsPerLane = 8;                       // outputs per lane
constexpr int kInsTile = kInsThreads * kInsPerLane;  // 2048 pixels
constexpr int kInsWindow = 1792;                     // bin lower edges per item
constexpr int kInsTapBlock = 256;                    // taps staged at once
// Doubles per plane: at least (tile + tap block) / 8, and 2 * stride = 16 mod
// 64 dwords, so that the 64 lanes of a staging write (8 planes x 8 rows) hit 64
// different bank pairs.
constexpr int kInsPlane = 296;
static_assert(8 * kInsPlane >= kInsTile + kInsTapBlock + 16, "staged block must fit");
static_assert((2 * kInsPlane) % 64 == 16, "planes must start on different banks");
static_assert(kInsMaxRatio + kInsWindow + 4 <= kInsTile, "bin span must fit the tile");
static_assert(kInsTapBlock % 16 == 0, "tap blocks are walked 16 at a time");

// A double that every lane of the wave holds alike, moved to scalar registers:
// FP64 arithmetic runs on the vector unit, so the skewer and tile constants
// would otherwise take a register pair in every lane for the whole walk.
__device__ inline double wave_uniform(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Per-skewer geometry shared by both kernels.
struct InsSkewer {
  int64_t off, n, out_off, n_out;
  double dv;       // pixel width, km/s
  double inv_dv;   // 1 / dv
  double q;        // bin width in pixels
  double inv_q;    // 1 / q
  int M;           // taps m = -M .. M
  bool half_ends;  // the two extreme taps are the same image (whole even box)
  bool ok;
};

__device__ InsSkewer ins_skewer(const InsArgs &a, int64_t s) {
  InsSkewer k;
  k.off = a.offsets[s];
  k.n = a.offsets[s + 1] - k.off;
  k.out_off = a.out_offsets[s];
  k.n_out = a.out_offsets[s + 1] - k.out_off;
  k.dv = wave_uniform((double)a.dv[s]);
  k.inv_dv = wave_uniform(1.0 / k.dv);
  k.q = wave_uniform(a.bin * k.inv_dv);
  k.inv_q = wave_uniform(k.dv * a.inv_bin);
  k.ok = k.dv > 0.0 && isfinite(k.dv) &&
         (k.n_out == 0 || (k.q <= (double)kInsMaxRatio &&
                           (double)k.n_out * a.bin <= (double)(int)k.n * k.dv * (1.0 + 1e-9)));
  k.M = 0;
  k.half_ends = false;
  if (a.fwhm > 0.0) {
    const double reach = a.window_k * a.fwhm * kInvTwoSqrtLn2 * k.inv_dv;  // k b_L / dv
    if (a.window_k > 0.0 && reach < 0.5 * (double)((int)k.n - 1)) {
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
  return __builtin_fma((double)bin, a.bin, a.v_start) * k.inv_dv + 0.5;
}

// i mod n in [0, n) for |i| < 2^52, 1 <= n <= 2^24 (a skewer's length).
__device__ inline int64_t wrap_index(int64_t i, int n) {
  int64_t r = i - (int64_t)floor((double)i / (double)n) * n;
  if (r < 0) r += n;
  if (r >= n) r -= n;
  return r;
}

// LDS of one workgroup.
struct InsShared {
  double s[8 * kInsPlane];  // staged values in 8 planes, later the prefix sums
  double h[kInsTapBlock];   // taps of the current block
  double red[kInsThreads / 64];
};

__device__ inline void stage_store(InsShared &sh, int x, double v) {
  sh.s[(x & 7) * kInsPlane + (x >> 3)] = v;
}

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

// The unnormalised tap at offset m, |m| <= M: g(m dv), halved at the two ends
// of a whole even box; scale = dv / b_L.
__device__ inline double tap_value(const InsArgs &a, const InsSkewer &k, int m, double scale) {
  if (!(a.fwhm > 0.0)) return 1.0;  // M = 0: the identity
  const double x = (double)m * scale;
  double g = exp(-x * x);
  if (k.half_ends && (m == k.M || m == -k.M)) g *= 0.5;
  return g;
}
__device__ inline double tap_scale(const InsArgs &a, const InsSkewer &k) {
  return a.fwhm > 0.0 ? k.dv / (a.fwhm * kInvTwoSqrtLn2) : 0.0;
}

// Taps u0 .. u0 + tbp - 1 of the walk (h_u = g((M - u) dv), zero past the tb
// real ones) into sh.h; returns this thread's share of their sum.
__device__ double stage_taps(const InsArgs &a, const InsSkewer &k, int u0, int tb, int tbp,
                             double *h) {
  double z_part = 0.0;
  const double scale = tap_scale(a, k);
  for (int u = threadIdx.x; u < tbp; u += kInsThreads) {
    const double g = u < tb ? tap_value(a, k, k.M - (u0 + u), scale) : 0.0;
    h[u] = g;
    z_part += g;
  }
  return z_part;
}

// Eight taps u .. u+7 against the window lo (elements 8l + u .. 8l + u + 7) and
// hi (the next 8).
__device__ inline void conv_step(int u, const double (&lo)[8], const double (&hi)[8],
                                 double (&acc)[kInsPerLane], const double *taps) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double h = taps[u + i];
#pragma unroll
    for (int q = 0; q < kInsPerLane; ++q)
      acc[q] = __builtin_fma(h, (q + i < 8) ? lo[q + i] : hi[q + i - 8], acc[q]);
  }
}

// acc[q] += sum_{u < tbp} h_u s[8l + q + u] over the staged block (tbp a
// multiple of 16): lane l owns outputs 8l .. 8l + 7; element 8l + 8b + j of the
// staged block sits in plane j at row l + b.
__device__ inline void conv_block(int tbp, double (&acc)[kInsPerLane], const InsShared &sh) {
  const double *p = sh.s + threadIdx.x;
  double wa[8], wb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) wa[j] = p[j * kInsPlane];
  for (int u = 0; u < tbp; u += 16) {
    const int b = u >> 3;
#pragma unroll
    for (int j = 0; j < 8; ++j) wb[j] = p[j * kInsPlane + b + 1];
    conv_step(u, wa, wb, acc, sh.h);
#pragma unroll
    for (int j = 0; j < 8; ++j) wa[j] = p[j * kInsPlane + b + 2];
    conv_step(u + 8, wb, wa, acc, sh.h);
  }
}

// Convolution of a tile: acc[q] = sum_{u < T} h_u src(8l + q + u) for the lane's
// outputs t = 8l + q < span, taps in blocks of kInsTapBlock (unnormalised; the
// sum of the taps is returned).  src(x) yields the value at staged offset x
// (x = 0 .. span + T - 2).
template <class Src>
__device__ double convolve_tile(const InsArgs &a, const InsSkewer &k, int span, Src src,
                                double (&acc)[kInsPerLane], InsShared &sh) {
  const int T = 2 * k.M + 1;
  const int tid = threadIdx.x;
  const bool wave_active = (tid & ~63) * kInsPerLane < span;
  double z_part = 0.0;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q) acc[q] = 0.0;
  for (int u0 = 0; u0 < T; u0 += kInsTapBlock) {
    const int tb = min(kInsTapBlock, T - u0);  // real taps in this block
    const int tbp = (tb + 15) & ~15;           // walked taps (zero-padded)
    __syncthreads();  // the previous block's readers are done
    z_part += stage_taps(a, k, u0, tb, tbp, sh.h);
    const int need = span + tbp - 1;  // staged offsets read by outputs < span
    const int real = span + tb - 1;   // offsets carrying real taps
    for (int x = tid; x < need; x += kInsThreads) stage_store(sh, x, x < real ? src(u0 + x) : 0.0);
    __syncthreads();
    if (wave_active) conv_block(tbp, acc, sh);
  }
  return block_sum_d(z_part, sh.red);
}

// Geometry of tile c of a skewer: the bins whose lower edge lies in pixels
// [c W, (c+1) W) from the first bin's edge, and the pixels they cover.
struct InsTile {
  int64_t k_lo, k_hi;  // bins k_lo .. k_hi - 1 (none if k_lo >= k_hi)
  int64_t p0;          // first pixel of the span (absolute; may lie outside [0, n))
  double e_lo;         // lower edge of bin k_lo relative to p0, pixels
  double xb;           // lower edge of bin k_hi, pixels
  uint32_t base;       // (p0 - M) mod n: pixel of staged offset 0
  int span;            // pixels covered
};

__device__ inline int64_t first_bin(const InsSkewer &k, int64_t c) {
  if (c == 0) return 0;
  if (c * kInsWindow >= k.n) return k.n_out;  // past the last tile
  // c kInsWindow < n, so kb <= n / q + 1, about n_out + 1: exact as int64
  const int64_t kb = (int64_t)ceil((double)(c * kInsWindow) * k.inv_q);
  return kb >= k.n_out ? k.n_out : kb;
}

// Tile c, given tile c - 1 (prev, for c > 0): the lower bin and edge of a tile
// are the upper ones of the one before, and its base moves with p0.
__device__ InsTile ins_tile(const InsArgs &a, const InsSkewer &k, int c, const InsTile *prev) {
  InsTile t;
  double xa;
  if (prev) {
    t.k_lo = prev->k_hi;
    xa = prev->xb;
  } else {
    t.k_lo = 0;
    xa = bin_edge(a, k, 0);
  }
  t.k_hi = first_bin(k, c + 1);
  t.p0 = 0;
  t.e_lo = 0.0;
  t.xb = xa;
  t.base = 0;
  t.span = 0;
  if (t.k_lo < t.k_hi) {
    t.xb = wave_uniform(bin_edge(a, k, t.k_hi));
    t.p0 = (int64_t)floor(xa);
    t.e_lo = wave_uniform(xa - (double)t.p0);
    t.span = (int)((int64_t)floor(t.xb) - t.p0 + 1);
    const int64_t step = prev ? t.p0 - prev->p0 : 0;  // 0 <= step <= kInsTile
    if (prev && step < k.n) {
      int64_t b = (int64_t)prev->base + step;
      if (b >= k.n) b -= k.n;
      t.base = (uint32_t)b;
    } else {
      t.base = (uint32_t)wrap_index(t.p0 - k.M, (int)k.n);
    }
  }
  return t;
}

constexpr int kNzPre = 4;  // noise draws per thread read ahead

// Staged offset x of a tile holds pixel (p0 - M + x) mod n; n <= 2^24, so 32
// bits do.
__device__ inline float tile_flux(const float *F, uint32_t n32, uint32_t base, int x) {
  uint32_t i = base + (uint32_t)x;
  if (i >= n32) i -= n32;
  if (i >= n32) i %= n32;
  return F[i];
}

// Thread t writes the bins j0 .. j0 + cnt - 1 of a tile (consecutive, so that
// neighbouring bins share the cumulative value at their common edge).
__device__ inline void bin_range(const InsTile &t, int &j0, int &cnt) {
  const int nb = (int)(t.k_hi - t.k_lo);
  const int cb = (nb + kInsThreads - 1) / kInsThreads;
  j0 = min((int)threadIdx.x * cb, nb);
  cnt = min(cb, nb - j0);
}

__device__ inline void noise_loads(const InsArgs &a, const InsSkewer &k, const InsTile &t,
                                   float (&nz)[kNzPre]) {
  int j0, cnt;
  bin_range(t, j0, cnt);
#pragma unroll
  for (int r = 0; r < kNzPre; ++r)
    nz[r] = (a.noise && r < cnt) ? a.noise[k.out_off + t.k_lo + j0 + r] : 0.0f;
}

// LDS of the forward when the taps fit one block: two buffers of the raw flux
// (FP32, 8 planes of kDmaRows rows: element x at plane x mod 8, row x / 8), the
// prefix sums of the convolved tile, the taps.
constexpr int kDmaRows = 320;  // 5 blocks of 64 rows
static_assert(8 * kDmaRows >= kInsTile + kInsTapBlock + 16, "a staged tile must fit");
struct InsDmaShared {
  float f[2][8 * kDmaRows];
  double pre[kInsTile + 8];
  double h[kInsTapBlock];
  double red[kInsThreads / 64];
};

// Staging of a tile straight from memory into LDS (global_load_lds: each lane's
// dword lands at the wave's LDS base + 4 lane), one wave instruction per plane
// and block of 64 rows, so no register holds it and the copy runs while the
// workgroup computes.  Offsets past the real taps load a pixel of the tile
// (they meet zero taps only).
__device__ inline void tile_dma(const float *F, uint32_t n32, const InsTile &t, int T, int tbp,
                                float *fbuf) {
  const int need = t.span + tbp - 1;
  const int real = t.span + T - 1;
  const int nrb = (((need + 7) >> 3) + 63) >> 6;  // blocks of 64 rows, <= 5
  const int lane = threadIdx.x & 63;
  for (int q = threadIdx.x >> 6; q < 8 * nrb; q += kInsThreads / 64) {
    const int j = q & 7, rb = q >> 3;
    const int x = 8 * (rb * 64 + lane) + j;
    uint32_t i = t.base + (uint32_t)(x < real ? x : 0);
    if (i >= n32) i -= n32;
    if (i >= n32) i %= n32;
    __builtin_amdgcn_global_load_lds(F + i, fbuf + j * kDmaRows + rb * 64, 4, 0, 0);
  }
}

// conv_block over a staged FP32 tile (each value converted once on load).
__device__ inline void conv_block_f32(int tbp, double (&acc)[kInsPerLane], const float *fbuf,
                                      const double *taps) {
  const float *p = fbuf + threadIdx.x;
  double wa[8], wb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) wa[j] = (double)p[j * kDmaRows];
  for (int u = 0; u < tbp; u += 16) {
    const int b = u >> 3;
#pragma unroll
    for (int j = 0; j < 8; ++j) wb[j] = (double)p[j * kDmaRows + b + 1];
    conv_step(u, wa, wb, acc, taps);
#pragma unroll
    for (int j = 0; j < 8; ++j) wa[j] = (double)p[j * kDmaRows + b + 2];
    conv_step(u + 8, wb, wa, acc, taps);
  }
}

// Prefix sums of a convolved tile, then its bins (with the noise draws nz read
// ahead for the first kNzPre of this thread's bins): each bin is the
// difference of the interpolated cumulative integral at its edges
// e(j) = e_lo + j q (relative to p0), divided by its width.
__device__ void finish_tile(const InsArgs &a, const InsSkewer &k, const InsTile &t,
                            const double (&acc)[kInsPerLane], double Z,
                            const float (&nz)[kNzPre], double *pre, double *red) {
  const int span = t.span;
  // pre[i] = sum_{i' < i} Fc[i']; only outputs inside the span enter (lanes
  // past it hold garbage)
  const double invZ = 1.0 / Z;
  const int t0 = threadIdx.x * kInsPerLane;
  double run = 0.0, loc[kInsPerLane];
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q) {
    if (t0 + q < span) run += acc[q] * invZ;
    loc[q] = run;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double incl = run;
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  __syncthreads();  // every wave is done with the staged values
  if (lane == 63) red[wv] = incl;
  __syncthreads();
  double excl = incl - run;
  for (int w = 0; w < wv; ++w) excl += red[w];
  if (threadIdx.x == 0) pre[0] = 0.0;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q)
    if (t0 + q < span) pre[t0 + q + 1] = excl + loc[q];
  __syncthreads();

  const auto cum = [&](double e) -> double {
    const int i = min((int)e, span - 1);
    const double f = e - (double)i;
    return __builtin_fma(f, pre[i + 1] - pre[i], pre[i]);
  };
  int j0, cnt;
  bin_range(t, j0, cnt);
  if (cnt <= 0) return;
  float *out = a.out + k.out_off + t.k_lo + j0;
  const float *noise = a.noise ? a.noise + k.out_off + t.k_lo + j0 : nullptr;
  double c0 = cum(__builtin_fma((double)j0, k.q, t.e_lo));
#pragma unroll
  for (int r = 0; r < kNzPre; ++r) {
    if (r < cnt) {
      const double c1 = cum(__builtin_fma((double)(j0 + r + 1), k.q, t.e_lo));
      out[r] = (float)__builtin_fma(c1 - c0, k.inv_q, a.sigma * (double)nz[r]);
      c0 = c1;
    }
  }
  for (int r = kNzPre; r < cnt; ++r) {
    const double c1 = cum(__builtin_fma((double)(j0 + r + 1), k.q, t.e_lo));
    out[r] = (float)__builtin_fma(c1 - c0, k.inv_q, a.sigma * (double)(noise ? noise[r] : 0.0f));
    c0 = c1;
  }
}

// Forward: one workgroup per skewer, walking its tiles in order.  When the
// taps fit one block (2M + 1 <= kInsTapBlock) the skewer's taps and their sum
// are formed once and the next tile's flux is copied into the other LDS buffer
// (and its noise draws read) while the current tile is convolved; wider
// line-spread functions stage the taps block by block for every tile.
union InsLds {
  InsShared w;     // wide line-spread functions
  InsDmaShared d;  // taps in one block
};

__global__ __launch_bounds__(kInsThreads) __attribute__((amdgpu_waves_per_eu(4))) void instrument_kernel(
    InsArgs a, const int2 *__restrict__ items) {
  __shared__ InsLds lds;
  const InsSkewer k = ins_skewer(a, items[blockIdx.x].x);
  if (!k.ok) {
    if (threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
    return;
  }
  const int T = 2 * k.M + 1;
  const float *F = a.in + k.off;
  const uint32_t n32 = (uint32_t)k.n;
  if (T > kInsTapBlock) {
    // a wider line-spread function: taps staged block by block for every tile
    InsShared &sh = lds.w;
    const int nt = (int)((k.n + kInsWindow - 1) / kInsWindow);
    InsTile t = ins_tile(a, k, 0, nullptr);
    for (int c = 0; c < nt && t.k_lo < t.k_hi; ++c) {
      if (t.span > kInsTile) {  // excluded by the bin-width limit; never expected
        if (threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
        return;
      }
      float nz[kNzPre];
      noise_loads(a, k, t, nz);
      const uint32_t base = t.base;
      const auto src = [&](int x) -> double { return (double)tile_flux(F, n32, base, x); };
      double acc[kInsPerLane];
      const double Z = convolve_tile(a, k, t.span, src, acc, sh);
      finish_tile(a, k, t, acc, Z, nz, sh.s, sh.red);
      const InsTile tn = ins_tile(a, k, c + 1, &t);
      t = tn;
    }
    return;
  }
  InsDmaShared &d = lds.d;
  const int tbp = (T + 15) & ~15;
  const int n_tiles = (int)((k.n + kInsWindow - 1) / kInsWindow);

  InsTile t = ins_tile(a, k, 0, nullptr);
  float nz[kNzPre];
  if (t.k_lo < t.k_hi && t.span <= kInsTile) tile_dma(F, n32, t, T, tbp, d.f[0]);
  noise_loads(a, k, t, nz);
  const double Z = block_sum_d(stage_taps(a, k, 0, T, tbp, d.h), d.red);

  for (int c = 0; c < n_tiles && t.k_lo < t.k_hi; ++c) {
    if (t.span > kInsTile) {  // excluded by the bin-width limit; never expected
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
      return;
    }
    // this tile's copy is complete for every wave
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // the next tile goes to the other buffer (last read by tile c - 1, whose
    // readers are past the barriers of its prefix sums) while this one computes
    const InsTile tn = ins_tile(a, k, c + 1, &t);
    const bool more = c + 1 < n_tiles && tn.k_lo < tn.k_hi && tn.span <= kInsTile;
    float nzn[kNzPre];
    if (more) {
      tile_dma(F, n32, tn, T, tbp, d.f[(c + 1) & 1]);
      noise_loads(a, k, tn, nzn);
    }
    double acc[kInsPerLane];
#pragma unroll
    for (int q = 0; q < kInsPerLane; ++q) acc[q] = 0.0;
    if ((int)(threadIdx.x & ~63u) * kInsPerLane < t.span)
      conv_block_f32(tbp, acc, d.f[c & 1], d.h);
    finish_tile(a, k, t, acc, Z, nz, d.pre, d.red);
    if (!(c + 1 < n_tiles && tn.k_lo < tn.k_hi)) break;
    t = tn;
#pragma unroll
    for (int j = 0; j < kNzPre; ++j) nz[j] = nzn[j];
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Adjoint of the binning for the cnt (<= 8) consecutive pixels i0 .. i0 + cnt
// - 1 of one image range: the gradient reaching each from the bins over it,
// overlap times the bin's gradient over the bin width, summed over the
// pixel's images that meet [x_first, x_last).  A merge walk: the current bin,
// its edges and its gradient carry from pixel to pixel, so each is formed
// once per run.  out(p, h) receives pixel i0 + p.
struct InsBinGeom {
  double x_first, x_last;  // lower edges of bin 0 and of bin n_out, pixels
  double nd, inv_nd;       // n and 1 / n
};
template <class GLoad, class Out>
__device__ inline void bin_adjoint_run(const InsArgs &a, const InsSkewer &k, const InsBinGeom &G,
                                       int64_t i0, int cnt, GLoad gload, Out out) {
  double acc[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p] = 0.0;
  // images y = i + L n of the run's pixels that meet the bins (a quotient
  // rounded across an integer only drops or adds an image whose overlap is
  // below 1e-9 px, or zero)
  const double L_lo = ceil((G.x_first - (double)(i0 + cnt - 1) - 1.0) * G.inv_nd);
  const double L_hi = floor((G.x_last - (double)i0) * G.inv_nd);
  for (double L = L_lo; L <= L_hi; L += 1.0) {
    const double y0 = (double)i0 + L * G.nd;
    int64_t kb = (int64_t)floor((y0 - G.x_first) * k.inv_q) - 1;
    if (kb < 0) kb = 0;
    if (kb >= k.n_out) continue;
    double e0 = bin_edge(a, k, kb), e1 = bin_edge(a, k, kb + 1);
    while (e1 <= y0 && kb + 1 < k.n_out) {  // to the first bin that ends past y0
      ++kb;
      e0 = e1;
      e1 = bin_edge(a, k, kb + 1);
    }
    double gk = (double)gload(kb) * k.inv_q;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p < cnt) {
        const double y = y0 + (double)p;
        while (kb < k.n_out && e0 < y + 1.0) {
          const double ov = fmin(y + 1.0, e1) - fmax(y, e0);
          if (ov > 0.0) acc[p] = __builtin_fma(ov, gk, acc[p]);
          if (e1 > y + 1.0) break;  // the bin continues into the next pixel
          if (++kb < k.n_out) {
            e0 = e1;
            e1 = bin_edge(a, k, kb + 1);
            gk = (double)gload(kb) * k.inv_q;
          }
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 8; ++p)
    if (p < cnt) out(p, acc[p]);
}

// LDS of the per-tile backward when the taps fit one block: the binning
// adjoint of the tile's staged pixels (FP32, planes as in the forward) and the
// taps.  That kernel takes the skewers with more than kInsBwdBins bins (read
// from memory) or none; the per-skewer kernel below takes the others.
constexpr int kInsBwdBins = 4096;
struct InsBwdShared {
  float f[8 * kDmaRows];
  double h[kInsTapBlock];
  double red[kInsThreads / 64];
};

union InsBwdLds {
  InsShared w;     // wide line-spread functions
  InsBwdShared d;  // taps in one block
};

// Backward: the adjoint of the binning at the tile's staged pixels, then the
// same line-spread convolution (the taps are even, so the adjoint convolves
// with them too).  Taps in one block: each thread forms the binning adjoint of
// eight consecutive staged pixels (one row of the eight planes) by the merge
// walk; wider line-spread functions form it pixel by pixel, block by block.
__global__ __launch_bounds__(kInsThreads) void instrument_backward_kernel(
    InsArgs a, const int2 *__restrict__ items) {
  __shared__ InsBwdLds lds;
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
  InsBinGeom G;
  G.nd = (double)(int)k.n;
  G.inv_nd = 1.0 / G.nd;
  G.x_first = bin_edge(a, k, 0);
  G.x_last = bin_edge(a, k, k.n_out);
  const float *g = a.in + k.out_off;
  const auto g_global = [&](int64_t kb) -> float { return g[kb]; };
  const uint32_t n32 = (uint32_t)k.n;
  const uint32_t base = (uint32_t)wrap_index(p0 - k.M, (int)k.n);
  const int T = 2 * k.M + 1;
  double acc[kInsPerLane];
  double Z;
  if (T <= kInsTapBlock) {
    InsBwdShared &d = lds.d;
    const int tbp = (T + 15) & ~15;
    const double z_part = stage_taps(a, k, 0, T, tbp, d.h);
    const int rows = (span + tbp - 1 + 7) >> 3;  // staged offsets read by outputs < span
    for (int r = threadIdx.x; r < rows; r += kInsThreads) {
      // staged offsets 8r .. 8r + 7 are pixels (base + x) mod n, consecutive
      // up to the end of the box
      uint32_t i = base + 8u * (uint32_t)r;
      if (i >= n32) i -= n32;
      if (i >= n32) i %= n32;
      int done = 0;
      while (done < 8) {
        const int c = min(8 - done, (int)(n32 - i));
        const int x0 = 8 * r + done;
        bin_adjoint_run(a, k, G, (int64_t)i, c, g_global, [&](int p, double v) {
          const int x = x0 + p;
          d.f[(x & 7) * kDmaRows + (x >> 3)] = (float)v;
        });
        done += c;
        i = 0;
      }
    }
    Z = block_sum_d(z_part, d.red);  // its barriers publish the staged values and the taps
#pragma unroll
    for (int q = 0; q < kInsPerLane; ++q) acc[q] = 0.0;
    if ((int)(threadIdx.x & ~63u) * kInsPerLane < span) conv_block_f32(tbp, acc, d.f, d.h);
  } else {
    const auto src = [&](int x) -> double {
      uint32_t i = base + (uint32_t)x;
      if (i >= n32) i -= n32;
      if (i >= n32) i %= n32;
      double v = 0.0;
      bin_adjoint_run(a, k, G, (int64_t)i, 1, g_global, [&](int, double h) { v = h; });
      return v;
    };
    Z = convolve_tile(a, k, span, src, acc, lds.w);
  }
  const double invZ = 1.0 / Z;
  const int t0 = threadIdx.x * kInsPerLane;
#pragma unroll
  for (int q = 0; q < kInsPerLane; ++q)
    if (t0 + q < span) gF[p0 + t0 + q] = (float)(acc[q] * invZ);
}

// Backward, one workgroup per skewer whose bins fit LDS (the per-tile kernel
// takes the skewers with more bins or none).  The binning adjoint of pixel
// [y, y + 1) (pixel coordinates, one image of the pixel) is C(y + 1) - C(y),
// where C is the integral of the bins' gradient density g_k / (bin width) from
// the first bin's lower edge, in pixel units: C = P[k] + t (P[k+1] - P[k]) at
// bin coordinate k + t (t in [0, 1); a pixel is 1 / q bin units, so the
// difference carries the 1 / q), with the prefix sums P[k] = sum_{k' < k} g_k'
// (C is 0 before the first bin and P[n_out] past the last), summed over the
// pixel's images that meet the bins.  P (FP64, n_out + 1 values, dynamic LDS)
// and the taps' sum are formed once; the skewer's tiles of kInsTile pixels are
// walked, each thread forming the adjoint of rows of eight staged pixels (tile
// + taps, FP32 in planes as in the per-tile kernel) and the tile convolved
// block of taps by block.  A wave whose staged window is all zero (pixels that
// no bin reaches within the taps) stores zeros without convolving.
struct InsBwdSkShared {
  float f[8 * kDmaRows];
  double h[kInsTapBlock];
  double red[kInsThreads / 64];
  double tot[kInsThreads / 64];
  uint8_t nz_row[kDmaRows];  // row r of the staged block holds a nonzero value
};
constexpr int kBwdPerThread = kInsBwdBins / kInsThreads;  // bins per thread in the prefix sums
static_assert(kBwdPerThread * kInsThreads == kInsBwdBins, "the prefix sums cover every bin");
static_assert(64 + kInsTapBlock / 8 <= 128, "a wave's staged rows are two per lane at most");
static_assert((kInsTile + kInsTapBlock) / 8 <= kInsThreads + kInsThreads / 8,
              "the staged rows past one per thread are at most one pixel per thread");

// Four waves per SIMD (at most 128 VGPRs), as many as the LDS of a skewer
// with up to ~2700 bins leaves room for.
__global__ __launch_bounds__(kInsThreads) __attribute__((amdgpu_waves_per_eu(4))) void
instrument_backward_skewer_kernel(InsArgs a, const int2 *__restrict__ items) {
  __shared__ InsBwdSkShared sh;
  extern __shared__ double P[];  // n_out + 1 prefix sums
  const InsSkewer k = ins_skewer(a, items[blockIdx.x].x);
  if (!k.ok) {
    if (threadIdx.x == 0) atomicOr(a.status, LYAF_STATUS_DOMAIN);
    return;
  }
  const int nb = (int)k.n_out;
  const float *g = a.in + k.out_off;
  // P[j + 1] = sum_{j' <= j} g_j': thread t sums bins 16t .. 16t + 15, then the
  // workgroup scans the threads' totals
  double v[kBwdPerThread];
  const int j0 = (int)threadIdx.x * kBwdPerThread;
#pragma unroll
  for (int j = 0; j < kBwdPerThread; ++j) v[j] = j0 + j < nb ? (double)g[j0 + j] : 0.0;
  const int T = 2 * k.M + 1;
  const bool one_block = T <= kInsTapBlock;
  // the taps' sum (and, when they fit one block, the taps themselves)
  double z_part = 0.0;
  if (one_block) {
    z_part = stage_taps(a, k, 0, T, (T + 15) & ~15, sh.h);
  } else {
    const double scale = tap_scale(a, k);
    for (int u = threadIdx.x; u < T; u += kInsThreads) z_part += tap_value(a, k, k.M - u, scale);
  }
#pragma unroll
  for (int j = 1; j < kBwdPerThread; ++j) v[j] += v[j - 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double incl = v[kBwdPerThread - 1];
  for (int d = 1; d < 64; d <<= 1) {
    const double o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  if (lane == 63) sh.tot[wv] = incl;
  double excl = __shfl_up(incl, 1);
  if (lane == 0) excl = 0.0;
  __syncthreads();
  for (int w = 0; w < wv; ++w) excl += sh.tot[w];
  if (threadIdx.x == 0) P[0] = 0.0;
#pragma unroll
  for (int j = 0; j < kBwdPerThread; ++j)
    if (j0 + j < nb) P[j0 + j + 1] = excl + v[j];
  const double invZ = 1.0 / block_sum_d(z_part, sh.red);  // its barriers publish P and the taps

  const double x_first = bin_edge(a, k, 0), x_last = bin_edge(a, k, k.n_out);
  const double nd = (double)(int)k.n, inv_nd = 1.0 / nd;
  const double Ptot = P[nb];
  const auto cum = [&](double y) -> double {
    const double t = (y - x_first) * k.inv_q;
    if (!(t > 0.0)) return 0.0;
    if (t >= (double)nb) return Ptot;
    const int kb = (int)t;
    return __builtin_fma(t - (double)kb, P[kb + 1] - P[kb], P[kb]);
  };
  const uint32_t n32 = (uint32_t)k.n;
  float *gF = a.out + k.off;
  const int n_tiles = (int)((k.n + kInsTile - 1) / kInsTile);
  bool first = true;  // no barrier owed to earlier readers of f and h
  for (int c = 0; c < n_tiles; ++c) {
    const int64_t p0 = (int64_t)c * kInsTile;
    const int span = (int)min<int64_t>(kInsTile, k.n - p0);
    const bool wave_active = (int)(threadIdx.x & ~63u) * kInsPerLane < span;
    double acc[kInsPerLane];
#pragma unroll
    for (int q = 0; q < kInsPerLane; ++q) acc[q] = 0.0;
    for (int u0 = 0; u0 < T; u0 += kInsTapBlock) {
      const int tb = min(kInsTapBlock, T - u0);  // real taps in this block
      const int tbp = (tb + 15) & ~15;           // walked taps (zero-padded)
      if (!first) __syncthreads();  // every wave is done with the previous block's values
      first = false;
      if (!one_block) stage_taps(a, k, u0, tb, tbp, sh.h);
      // staged offset x is pixel (p0 - M + u0 + x) mod n
      const uint32_t base = (uint32_t)wrap_index(p0 - k.M + u0, (int)k.n);
      const int rows = (span + tbp - 1 + 7) >> 3;  // staged offsets read by outputs < span
      // the gathered gradients of cnt consecutive pixels from pixel i (no wrap
      // inside the run), at staged offsets x0 .. x0 + cnt - 1; true if any is
      // nonzero
      const auto gather = [&](const uint32_t i, const int cnt, const int x0) -> bool {
        double G[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) G[p] = 0.0;
        // images y = i + L n of the run's pixels that meet [x_first, x_last)
        const double L_lo = ceil((x_first - (double)(i + cnt - 1) - 1.0) * inv_nd);
        const double L_hi = floor((x_last - (double)i) * inv_nd);
        for (double L = L_lo; L <= L_hi; L += 1.0) {
          const double y0 = __builtin_fma(L, nd, (double)i);
          double c0 = cum(y0);
#pragma unroll
          for (int p = 0; p < 8; ++p) {
            if (p < cnt) {
              const double c1 = cum(y0 + (double)(p + 1));
              G[p] += c1 - c0;
              c0 = c1;
            }
          }
        }
        bool any = false;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          if (p < cnt) {
            const int x = x0 + p;
            const float gv = (float)G[p];
            any |= gv != 0.0f;
            sh.f[(x & 7) * kDmaRows + (x >> 3)] = gv;
          }
        }
        return any;
      };
      const auto wrap_px = [&](uint32_t i) {
        if (i >= n32) i -= n32;
        if (i >= n32) i %= n32;
        return i;
      };
      // staged offsets 8r .. 8r + 7 (pixels consecutive up to the end of the
      // box) for the first kInsThreads rows, one row per thread; the rows past
      // those (rows <= kInsThreads + kInsTapBlock / 8) one pixel per thread, so
      // that no thread gathers two rows while the others wait at the barrier
      if ((int)threadIdx.x < rows) {
        const int r = threadIdx.x;
        uint32_t i = wrap_px(base + 8u * (uint32_t)r);
        int done = 0;
        bool any = false;
        while (done < 8) {  // a box shorter than the row wraps more than once
          const int cnt = min(8 - done, (int)(n32 - i));
          any |= gather(i, cnt, 8 * r + done);
          done += cnt;
          i = 0;
        }
        sh.nz_row[r] = any ? 1 : 0;
      }
      if (rows > kInsThreads) {
        const int x = 8 * kInsThreads + (int)threadIdx.x;  // one pixel
        const bool in = x < 8 * rows;
        const bool nz = in && gather(wrap_px(base + (uint32_t)x), 1, x);
        // a row's 8 pixels sit on 8 consecutive lanes of one wave
        const uint64_t bal = __ballot(nz);
        if (in && (lane & 7) == 0) sh.nz_row[x >> 3] = ((bal >> (lane & ~7)) & 0xFFu) ? 1 : 0;
      }
      __syncthreads();
      // rows 64 w .. 64 w + 63 + tbp / 8 feed wave w's outputs
      const int r0 = (int)(threadIdx.x & ~63u) + lane;
      const int r1 = r0 + 64;
      const bool mine = (r0 < rows && sh.nz_row[r0]) ||
                        (lane <= tbp / 8 - 1 && r1 < rows && sh.nz_row[r1]);
      if (wave_active && __any(mine)) conv_block_f32(tbp, acc, sh.f, sh.h);
    }
    const int t0 = threadIdx.x * kInsPerLane;
#pragma unroll
    for (int q = 0; q < kInsPerLane; ++q)
      if (t0 + q < span) gF[p0 + t0 + q] = (float)(acc[q] * invZ);
  }
}

}  // namespace

bool ins_bwd_skewer_item(int64_t n, int64_t n_out) {
  return n > 0 && n_out > 0 && n_out <= kInsBwdBins;
}

int ins_items_per_skewer(int64_t n, int64_t n_out, bool backward) {
  if (n <= 0) return 0;
  if (backward)  // skewers with 1 .. kInsBwdBins bins go to the per-skewer kernel
    return ins_bwd_skewer_item(n, n_out) ? 0 : (int)((n + kInsTile - 1) / kInsTile);
  return n_out > 0 ? 1 : 0;  // the forward takes a whole skewer per workgroup
}

hipError_t launch_instrument(const InsArgs &a, const int2 *items, int64_t n_items,
                             const int2 *skewer_items, int64_t n_skewer_items, int max_bins,
                             bool backward, hipStream_t st) {
  if (backward) {
    // each skewer is taken by exactly one of the two kernels
    if (n_skewer_items > 0)
      hipLaunchKernelGGL(instrument_backward_skewer_kernel, dim3((unsigned)n_skewer_items),
                         dim3(kInsThreads), sizeof(double) * (size_t)(max_bins + 1), st, a,
                         skewer_items);
    if (n_items > 0)
      hipLaunchKernelGGL(instrument_backward_kernel, dim3((unsigned)n_items), dim3(kInsThreads),
                         0, st, a, items);
  } else if (n_items > 0) {
    hipLaunchKernelGGL(instrument_kernel, dim3((unsigned)n_items), dim3(kInsThreads), 0, st, a,
                       items);
  }
  return hipGetLastError();
}

}  // namespace lyaf
