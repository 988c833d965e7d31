// lyaf_tau.hip -- optical-depth kernels for gfx950 (Greig, Bolton & Wyithe 2011,
// Section 2.3, eqs. 4-6).
//
//   reach_kernel        one workgroup per skewer: per-skewer constants in FP64,
//                       the largest velocity-space reach (|v_j| + k b_j) / dv in
//                       pixels, and the device-side domain checks.
//   tau_window_kernel   one workgroup per 256-pixel target tile.  The sources
//                       that can reach the tile (tile +- reach) are staged once
//                       into LDS as (w, r, v, a, Q) plus the window bounds of
//                       every 16-source group.  Each wave splits into S source
//                       streams of 64/S lanes; a lane owns M consecutive
//                       targets and, per source, evaluates the first Gaussian
//                       with one exp2 and the other M-1 with the exact
//                       recurrence E_{k+1} = E_k R_k, R_{k+1} = R_k Q (the
//                       exponent of eq. 6 is quadratic in the target index).
//                       Streams sum in FP32 with a blocked Kahan fold and meet
//                       in a butterfly across lanes at the end.
//                       Short or very wide skewers (tile + 2 reach > N) take a
//                       full-sum path over every source with the minimal
//                       periodic image chosen per pair.
//   tau_plain_kernel    the literal full O(N^2) sum, one thread per target,
//                       naive FP32 accumulation (the comparison baseline).
#include <math.h>

#include "lyaf_internal.h"

namespace lyaf {

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }

// Per-source quantities from eqs. (4)-(5), FP32, log domain.
//   w = W Delta^2 D^(-1.2 (gamma-1)),  r = sqrt(log2 e)/b = R D^(-(gamma-1)/2),
//   b = B D^((gamma-1)/2),  D = min(Delta, pivot).
struct Src {
  float w, r, b;
};
__device__ __forceinline__ Src source_of(float delta, const SkewerConst &K, float pivot) {
  Src o;
  if (delta > 0.f) {
    const float D = fmaxf(fminf(delta, pivot), 1e-30f);
    const float x = K.gm1 * flog2(D);
    o.w = K.W * delta * delta * fexp2(kTempExpW * x);
    o.r = K.R * fexp2(kTempExpR * x);
    o.b = K.B * fexp2(0.5f * x);
  } else {  // empty pixel: no neutral hydrogen (the Delta -> 0 limit of eq. 4)
    o.w = 0.f;
    o.r = K.R;
    o.b = 0.f;
  }
  return o;
}

template <typename T>
__device__ __forceinline__ T block_reduce_max(T v, T *sh) {
  for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) v = fmaxf(v, sh[k]);
    sh[0] = v;
  }
  __syncthreads();
  return sh[0];
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reach_kernel(Batch b) {
  __shared__ float shm[8];
  __shared__ int shbad[1];
  const int64_t s = blockIdx.x;
  const int64_t off = b.offsets[s];
  const int n = (int)(b.offsets[s + 1] - off);
  const float dv = b.dv[s], T0 = b.T0[s], gm = b.gamma[s];
  int bad = !(dv > 0.f) || !isfinite(dv) || !(T0 > 0.f) || !isfinite(T0) || !isfinite(gm);
  if (threadIdx.x == 0) shbad[0] = 0;
  __syncthreads();
  // per-skewer constants, FP64, rounded once
  SkewerConst K;
  {
    const double T0d = bad ? 1e4 : (double)T0, dvd = bad ? 1.0 : (double)dv;
    const double sq = sqrt(T0d);
    K.W = (float)((double)b.tau_ref * pow(1e4, 0.7) * dvd / (kSqrtPi * kBeta) *
                  pow(T0d, -1.2));
    K.R = (float)(kSqrtLog2e / (kBeta * sq));
    K.B = (float)(kBeta * sq);
    K.gm1 = bad ? 0.f : gm - 1.f;
    K.dv = (float)dvd;
    K.inv_dv = (float)(1.0 / dvd);
    K.n = n;
  }
  float mr = 0.f;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const float d = b.delta[off + j], v = b.vpec[off + j];
    if (!(d >= 0.f) || !isfinite(d) || !isfinite(v)) bad = 1;
    if (d > 0.f) {
      const Src o = source_of(d, K, b.pivot);
      mr = fmaxf(mr, (fabsf(v) + b.window_k * o.b) * K.inv_dv);
    }
  }
  if (bad) atomicOr(shbad, 1);
  mr = block_reduce_max(mr, shm);
  if (threadIdx.x == 0) {
    int R = n;
    if (b.window_k > 0.f && mr < 1e8f) R = min(n, (int)ceilf(mr) + 2);
    K.reach = R;
    b.skc[s] = K;
    if (shbad[0]) atomicOr(b.status, LYAF_STATUS_DOMAIN);
  }
}

hipError_t launch_reach(const Batch &b, hipStream_t st) {
  if (b.n_skewers == 0) return hipSuccess;
  hipLaunchKernelGGL(reach_kernel, dim3((unsigned)b.n_skewers), dim3(256), 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Full sum over every source of the skewer with the minimal periodic image
// chosen per pair; one target per thread.  COMP selects the blocked Kahan fold.
template <bool COMP>
__device__ void full_sum_tile(const Batch &b, const SkewerConst &K, int64_t off, int i0,
                              float *__restrict__ tau, float4 *rec) {
  const int n = K.n;
  const int i = i0 + (int)threadIdx.x;
  const float dv = K.dv;
  const float nf = (float)n;
  const float invV = 1.f / (nf * dv);
  float sum = 0.f, comp = 0.f, blk = 0.f;
  for (int c0 = 0; c0 < n; c0 += kChunk) {
    const int cnt = min(kChunk, n - c0);
    __syncthreads();
    for (int c = threadIdx.x; c < cnt; c += blockDim.x) {
      const int j = c0 + c;
      const float d = b.delta[off + j], v = b.vpec[off + j];
      const Src o = source_of(d, K, b.pivot);
      rec[c] = make_float4(o.w, o.r, v, 0.f);
    }
    __syncthreads();
    float fd = (float)(i - c0);
    for (int c = 0; c < cnt; ++c) {
      const float4 q = rec[c];
      const float d0 = __builtin_fmaf(fd, dv, -q.z);
      const float img = floorf(__builtin_fmaf(d0, invV, 0.5f));
      const float fd2 = __builtin_fmaf(img, -nf, fd);  // exact: integers below 2^24
      const float d = __builtin_fmaf(fd2, dv, -q.z);
      const float t = d * q.y;
      blk = __builtin_fmaf(q.x, fexp2(-(t * t)), blk);
      fd -= 1.f;
      if (COMP && (c & 15) == 15) {
        const float y = blk - comp;
        const float tt = sum + y;
        comp = (tt - sum) - y;
        sum = tt;
        blk = 0.f;
      }
    }
  }
  if (COMP) {
    const float y = blk - comp;
    const float tt = sum + y;
    comp = (tt - sum) - y;
    sum = tt;
    sum -= comp;
  } else {
    sum = blk;
  }
  if (i < n) tau[off + i] = sum;
}

// Windowed tile.  S source streams per wave, M consecutive targets per lane.
template <int S, int M, bool DIRECT>
__global__ __launch_bounds__(kTauThreads) void tau_window_kernel(Batch b,
                                                                 const int2 *__restrict__ items,
                                                                 float *__restrict__ tau) {
  constexpr int L = kWave / S;           // lanes per stream
  constexpr int Tt = L * M;              // targets per wave sub-tile
  constexpr int NW = kTauThreads / kWave;
  constexpr int SUB = kTauTile / (NW * Tt);
  static_assert(SUB * NW * Tt == kTauTile, "tile shape");
  static_assert(kGroup % S == 0, "streams must divide a group");
  constexpr int KB = 16;                 // Kahan fold period (sources per stream)

  __shared__ float4 rec[kChunk];
  __shared__ float qrec[kChunk];
  __shared__ float2 bnd[kChunk / kGroup];
  __shared__ int gcold[kChunk / kGroup];

  const int2 item = items[blockIdx.x];
  const int64_t s = item.x;
  const int i0 = item.y * kTauTile;
  const SkewerConst K = b.skc[s];
  const int64_t off = b.offsets[s];
  const int n = K.n;
  const int R = K.reach;

  int e_lo = i0 - R;
  e_lo = (e_lo >= 0) ? (e_lo / kGroup) * kGroup : -(((-e_lo) + kGroup - 1) / kGroup) * kGroup;
  int e_hi = i0 + kTauTile + R;
  e_hi = ((e_hi + kGroup - 1) / kGroup) * kGroup;
  const int cnt = e_hi - e_lo;
  if (cnt > n || cnt > kChunk) {  // the window covers the box: full sum
    full_sum_tile<true>(b, K, off, i0, tau, rec);
    return;
  }

  // ---- stage sources e_lo .. e_hi-1 (extended, periodic) with group bounds
  const float pivot = b.pivot, wk = b.window_k;
  for (int c = threadIdx.x; c < cnt; c += kTauThreads) {
    const int e = e_lo + c;
    const int j = e < 0 ? e + n : (e >= n ? e - n : e);
    const float d = b.delta[off + j], v = b.vpec[off + j];
    const Src o = source_of(d, K, pivot);
    float lo = INFINITY, hi = -INFINITY;
    if (o.w > 0.f) {
      const float cc = (float)e + v * K.inv_dv;  // line centre, extended pixels
      const float h = wk * o.b * K.inv_dv;       // half window, pixels
      lo = cc - h;
      hi = cc + h;
    }
    const float a = K.dv * o.r;  // step of t = d r per target pixel
    rec[c] = make_float4(o.w, o.r, v, a);
    qrec[c] = fexp2(-2.f * a * a);
    // an unresolved line (b < 1.2 dv) makes the recurrence's dynamic range
    // too wide for FP32: its group is evaluated with one exp per pair
    int cold = (o.w > 0.f && a > kRecurrenceMaxStep) ? 1 : 0;
    for (int m = 1; m < kGroup; m <<= 1) {
      lo = fminf(lo, __shfl_xor(lo, m));
      hi = fmaxf(hi, __shfl_xor(hi, m));
      cold |= __shfl_xor(cold, m);
    }
    if ((threadIdx.x & (kGroup - 1)) == 0) {
      bnd[c / kGroup] = make_float2(lo, hi);
      gcold[c / kGroup] = cold;
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int sl = lane % S;   // stream
  const int ll = lane / S;   // lane within the stream
  const int ngroups = cnt / kGroup;
  const float dv = K.dv;

  for (int qsub = 0; qsub < SUB; ++qsub) {
    const int t0 = i0 + (qsub * NW + wave) * Tt;
    if (t0 >= n) break;
    const float tlo = (float)t0 - 1.f, thi = (float)(t0 + Tt) + 1.f;
    bool hit0 = false, hit1 = false, cold0 = false, cold1 = false;
    if (lane < ngroups) {
      const float2 bb = bnd[lane];
      hit0 = bb.y >= tlo && bb.x <= thi;
      cold0 = gcold[lane] != 0;
    }
    if (lane + kWave < ngroups) {
      const float2 bb = bnd[lane + kWave];
      hit1 = bb.y >= tlo && bb.x <= thi;
      cold1 = gcold[lane + kWave] != 0;
    }
    const uint64_t m0 = __ballot(hit0), m1 = __ballot(hit1);
    const uint64_t cm0 = __ballot(cold0), cm1 = __ballot(cold1);
    const int tb = t0 + ll * M;  // first target of this lane
    float sum[M], comp[M], blk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) sum[k] = comp[k] = blk[k] = 0.f;

    if (m0 | m1) {
      const int gfirst = m0 ? __builtin_ctzll(m0) : kWave + __builtin_ctzll(m1);
      const int glast = m1 ? 2 * kWave - 1 - __builtin_clzll(m1) : kWave - 1 - __builtin_clzll(m0);
      float fd = (float)(tb - (e_lo + gfirst * kGroup + sl));  // target - source, exact
      int since = 0;
      for (int g = gfirst; g <= glast; ++g) {
        const bool gc = ((g < kWave ? (cm0 >> g) : (cm1 >> (g - kWave))) & 1ull) != 0;
#pragma unroll
        for (int u = 0; u < kGroup / S; ++u) {
          const int c = g * kGroup + u * S + sl;
          const float4 q = rec[c];
          const float w = q.x, r = q.y, v = q.z;
          if (DIRECT || gc) {
#pragma unroll
            for (int k = 0; k < M; ++k) {
              const float d = __builtin_fmaf(fd + (float)k, dv, -v);
              const float t = d * r;
              blk[k] = __builtin_fmaf(w, fexp2(-(t * t)), blk[k]);
            }
          } else {
            const float a = q.w, Q = qrec[c];
            const float d0 = __builtin_fmaf(fd, dv, -v);
            const float t0v = d0 * r;
            float E = fexp2(-(t0v * t0v));
            // With a <= 1 the clamp only acts where E_0 is already 0 in FP32 and
            // the later terms are below 2^-85 of the line peak; it keeps
            // 0 * inf out of the recurrence.
            float Rk = fexp2(fminf(-(a * __builtin_fmaf(2.f, t0v, a)), 64.f));
            blk[0] = __builtin_fmaf(w, E, blk[0]);
#pragma unroll
            for (int k = 1; k < M; ++k) {
              E *= Rk;
              blk[k] = __builtin_fmaf(w, E, blk[k]);
              if (k + 1 < M) Rk *= Q;
            }
          }
          fd -= (float)S;
        }
        if (++since == KB / (kGroup / S)) {
          since = 0;
#pragma unroll
          for (int k = 0; k < M; ++k) {
            const float y = blk[k] - comp[k];
            const float tt = sum[k] + y;
            comp[k] = (tt - sum[k]) - y;
            sum[k] = tt;
            blk[k] = 0.f;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const float y = blk[k] - comp[k];
        const float tt = sum[k] + y;
        comp[k] = (tt - sum[k]) - y;
        sum[k] = tt - comp[k];
      }
      // butterfly over the S streams that share these targets
#pragma unroll
      for (int m = 1; m < S; m <<= 1) {
#pragma unroll
        for (int k = 0; k < M; ++k) sum[k] += __shfl_xor(sum[k], m);
      }
    }
    if (sl == 0) {
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (tb + k < n) tau[off + tb + k] = sum[k];
    }
  }
}

hipError_t launch_tau_window(const Batch &b, const int2 *items, int64_t n_items, float *tau,
                             bool direct, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  if (direct)
    hipLaunchKernelGGL((tau_window_kernel<16, 4, true>), dim3((unsigned)n_items),
                       dim3(kTauThreads), 0, st, b, items, tau);
  else
    hipLaunchKernelGGL((tau_window_kernel<16, 4, false>), dim3((unsigned)n_items),
                       dim3(kTauThreads), 0, st, b, items, tau);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTauThreads) void tau_plain_kernel(Batch b, int64_t s,
                                                                float *__restrict__ tau) {
  __shared__ float4 rec[kChunk];
  const SkewerConst K = b.skc[s];
  full_sum_tile<false>(b, K, b.offsets[s], (int)blockIdx.x * kTauThreads, tau, rec);
}

hipError_t launch_tau_plain(const Batch &b, int64_t skewer, int64_t n, float *tau,
                            hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(tau_plain_kernel, dim3((unsigned)((n + kTauThreads - 1) / kTauThreads)),
                     dim3(kTauThreads), 0, st, b, skewer, tau);
  return hipGetLastError();
}

}  // namespace lyaf
