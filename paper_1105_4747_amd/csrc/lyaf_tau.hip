// lyaf_tau.hip -- optical-depth kernels for gfx950 (Greig, Bolton & Wyithe 2011,
// Section 2.3, eqs. 4-6).
//
//   reach_kernel        one workgroup per skewer: per-skewer constants in FP64,
//                       the largest velocity-space reach (|v_j| + k b_j) / dv in
//                       pixels, and the device-side domain checks.
//   tau_skew_kernel     one workgroup per tile of 1024 (or 512, or 2048)
//                       targets; with the recurrence below over 4 targets per
//                       lane, the default shape.  The sources that can reach the tile
//                       (tile +- reach) are staged once into LDS as
//                       (w, r, v, a = dv r), or (w, a, v r, C) for the
//                       recurrence, in four planes by index mod 4,
//                       with each source's window bounds.  A lane owns 4
//                       consecutive targets and walks its own run of sources,
//                       shifted with its targets, whose start and length are
//                       uniform over the wave and come from the window bounds
//                       of the sources that meet the wave's 256 targets.  Per
//                       source and lane: one exact FMA for the velocity
//                       offset, one exp2 per pair, FP32 sums in three levels
//                       (blocks of 16 terms, partial sums of 8 blocks, their
//                       sum); no cross-lane reduction.
//   tau_window_kernel   the earlier shared-run form: a wave splits into S
//                       source streams that share a sub-tile of 64 M / S
//                       targets, visits the contiguous run of source groups
//                       whose windows reach it, and sums the streams in a DPP
//                       butterfly.
//   Short or very wide skewers (tile + 2 reach > N) take a full-sum path over
//   every source with the minimal periodic image chosen per pair.
//   tau_plain_kernel    the literal full O(N^2) sum, one thread per target,
//                       naive FP32 accumulation (the comparison baseline).
#include <math.h>

#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

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

// Sticky domain bit when any lane of the wave has read an invalid density
// (negative or not finite).  Every kernel that stages sources checks them: the
// reach pass reads Delta only when the temperature-density relation needs it.
__device__ __forceinline__ void flag_bad_delta(const Batch &b, bool bad) {
  if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(b.status, LYAF_STATUS_DOMAIN);
}
__device__ __forceinline__ bool bad_delta(float d) { return !(d >= 0.f) || !isfinite(d); }

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
    const double R = kSqrtLog2e / (kBeta * sq);
    K.R = (float)R;
    // a line's integral over the pixels goes as w / r, so W is rounded
    // together with the rounding of R: W / R is then off by one rounding
    K.W = (float)((double)b.tau_ref * pow(1e4, 0.7) * dvd / (kSqrtPi * kBeta) *
                  pow(T0d, -1.2) * ((double)K.R / R));
    K.B = (float)(kBeta * sq);
    K.gm1 = bad ? 0.f : gm - 1.f;
    K.dv = (float)dvd;
    K.inv_dv = (float)(1.0 / dvd);
    K.n = n;
  }
  float mr = 0.f;
  if (!bad && K.gm1 >= 0.f && isfinite(b.pivot)) {
    // T rises with Delta up to the pivot, so b <= beta sqrt(T0 pivot^(gamma-1))
    // for every source: only the velocities are read.  The kernels that stage
    // the sources check Delta.
    const float b_piv =
        (float)(kBeta * sqrt((double)T0 * pow((double)b.pivot, (double)K.gm1)) * (1.0 + 1e-6));
    float mv = 0.f;
    const float *vp = b.vpec + off;
    auto one = [&](const float v) {
      mv = fmaxf(mv, fabsf(v));
      if (!isfinite(v)) bad = 1;
    };
    // float4 reads from the first 16-byte boundary, four in flight per thread
    // (a 4096-pixel skewer in one round); the few values before and after
    // are read one by one
    const int head =
        (int)min<int64_t>(n, (int64_t)(((16u - (reinterpret_cast<uintptr_t>(vp) & 15u)) & 15u) >> 2));
    const int n4 = (n - head) >> 2;
    const float4 *v4 = reinterpret_cast<const float4 *>(vp + head);
    const int bd = (int)blockDim.x;
    int j = threadIdx.x;
    for (; j + 3 * bd < n4; j += 4 * bd) {
      float4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = v4[j + u * bd];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        one(q[u].x);
        one(q[u].y);
        one(q[u].z);
        one(q[u].w);
      }
    }
    for (; j < n4; j += bd) {
      const float4 q = v4[j];
      one(q.x);
      one(q.y);
      one(q.z);
      one(q.w);
    }
    if ((int)threadIdx.x < head) one(vp[threadIdx.x]);
    for (int t = head + 4 * n4 + (int)threadIdx.x; t < n; t += bd) one(vp[t]);
    if (n > 0) mr = (mv + b.window_k * b_piv) * K.inv_dv;
  } else {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const float d = b.delta[off + j], v = b.vpec[off + j];
      if (!(d >= 0.f) || !isfinite(d) || !isfinite(v)) bad = 1;
      if (d > 0.f) {
        const Src o = source_of(d, K, b.pivot);
        mr = fmaxf(mr, (fabsf(v) + b.window_k * o.b) * K.inv_dv);
      }
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
    bool bad = false;
    for (int c = threadIdx.x; c < cnt; c += blockDim.x) {
      const int j = c0 + c;
      const float d = b.delta[off + j], v = b.vpec[off + j];
      bad |= bad_delta(d);
      const Src o = source_of(d, K, b.pivot);
      rec[c] = make_float4(o.w, o.r, v, 0.f);
    }
    flag_bad_delta(b, bad);
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

// Lane permutations inside a row of 16 lanes (DPP), used to sum over the
// source streams that share a set of targets.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7-i within each 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15-i within each 16 lanes

template <int S>
__device__ __forceinline__ float stream_sum(float x) {
  static_assert(S == 4 || S == 8 || S == 16, "streams");
  x += dpp<kDppXor1>(x);
  x += dpp<kDppXor2>(x);
  if (S >= 8) x += dpp<kDppHalfMirror>(x);
  if (S >= 16) x += dpp<kDppMirror>(x);
  return x;
}
template <int S>
__device__ __forceinline__ float stream_min(float x) {
  x = fminf(x, dpp<kDppXor1>(x));
  x = fminf(x, dpp<kDppXor2>(x));
  if (S >= 8) x = fminf(x, dpp<kDppHalfMirror>(x));
  if (S >= 16) x = fminf(x, dpp<kDppMirror>(x));
  return x;
}
template <int S>
__device__ __forceinline__ float stream_max(float x) {
  x = fmaxf(x, dpp<kDppXor1>(x));
  x = fmaxf(x, dpp<kDppXor2>(x));
  if (S >= 8) x = fmaxf(x, dpp<kDppHalfMirror>(x));
  if (S >= 16) x = fmaxf(x, dpp<kDppMirror>(x));
  return x;
}

// Windowed tile of kTauTile targets.  A wave is S source streams of L = 64/S
// lanes; a lane owns M consecutive targets, so the streams of a wave share a
// sub-tile of L*M targets and one loop iteration evaluates S sources (one
// bounds group) against it.  The wave visits only the contiguous run of groups
// whose windows reach the sub-tile, then the streams' partial sums meet in a
// DPP butterfly.  Per source and lane: d0 = (i - j) dv - v_j exactly (one FMA
// on the integer offset), t_k = t_0 + k a_j (a_j = dv r_j),
// E_k = exp2(-t_k^2), acc_k += w_j E_k.
template <int S, int M, int TILE>
__device__ __forceinline__ void tau_tile(const Batch &b, const int2 item, float *__restrict__ tau,
                                         float4 *rec, float2 *bnd) {
  constexpr int G = S;                   // sources per bounds group = streams
  constexpr int L = kWave / S;           // lanes per stream
  constexpr int Tt = L * M;              // targets per wave sub-tile
  constexpr int NW = kTauThreads / kWave;
  constexpr int SUB = TILE / (NW * Tt);
  constexpr int NG = kChunk / G;
  static_assert(SUB * NW * Tt == TILE, "tile shape");
  constexpr int KB = 16;                 // Kahan fold period (sources per stream)

  const int64_t s = item.x;
  const int i0 = item.y * TILE;
  const SkewerConst K = b.skc[s];
  const int64_t off = b.offsets[s];
  const int n = K.n;
  const int R = K.reach;
  const int i_end = min(i0 + TILE, n);

  // staged sources: extended (periodic) indices e_lo .. e_hi-1.  A short
  // skewer appears together with its images; every sub-tile's run of sources
  // stays shorter than the skewer, so no source is counted twice.
  int e_lo = i0 - R;
  e_lo = (e_lo >= 0) ? (e_lo / G) * G : -(((-e_lo) + G - 1) / G) * G;
  int e_hi = i_end + R;
  e_hi = ((e_hi + G - 1) / G) * G;
  const int cnt = e_hi - e_lo;
  if (Tt + 2 * R + 3 * G > n || cnt > kChunk) {  // the window covers the box
    for (int q = i0; q < i_end; q += kTauThreads)
      full_sum_tile<true>(b, K, off, q, tau, rec);
    return;
  }

  const float pivot = b.pivot, wk = b.window_k;
  bool bad = false;
  for (int c = threadIdx.x; c < cnt; c += kTauThreads) {
    const int e = e_lo + c;  // -n < e < 2n in window mode (R < n/2)
    const int j = e < 0 ? e + n : (e >= n ? e - n : e);
    const float d = b.delta[off + j], v = b.vpec[off + j];
    bad |= bad_delta(d);
    const Src o = source_of(d, K, pivot);
    float lo = INFINITY, hi = -INFINITY;
    if (o.w > 0.f) {
      const float cc = __builtin_fmaf(v, K.inv_dv, (float)e);  // line centre, pixels
      const float h = wk * o.b * K.inv_dv;                     // half window, pixels
      lo = cc - h;
      hi = cc + h;
    }
    rec[c] = make_float4(o.w, o.r, v, K.dv * o.r);
    lo = stream_min<G>(lo);
    hi = stream_max<G>(hi);
    if ((threadIdx.x & (G - 1)) == 0) bnd[c / G] = make_float2(lo, hi);
  }
  flag_bad_delta(b, bad);
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform values live in scalar registers: the sub-tile loop and the
  // group scan then need no execution-mask bookkeeping
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int sl = lane & (S - 1);  // stream
  const int ll = lane / S;        // lane within the stream
  const int ngroups = cnt / G;
  const float dv = K.dv;

  for (int qsub = 0; qsub < SUB; ++qsub) {
    const int t0 = __builtin_amdgcn_readfirstlane(i0 + (qsub * NW + wave) * Tt);
    if (t0 >= i_end) break;
    // contiguous run of groups whose windows reach [t0, t0 + Tt): only groups
    // within the reach of the sub-tile can, so one ballot usually covers them
    const float tlo = (float)t0 - 1.f, thi = (float)(t0 + Tt) + 1.f;
    const int gs = max(0, (t0 - R - e_lo) / G - 1);
    const int ge = min(ngroups - 1, (t0 + Tt + R - e_lo) / G + 1);
    int gfirst = NG, glast = -1;
    for (int gb = gs; gb <= ge; gb += kWave) {
      const int g = gb + lane;
      bool hit = false;
      if (g <= ge) {
        const float2 bb = bnd[g];
        hit = bb.y >= tlo && bb.x <= thi;
      }
      const uint64_t m = __ballot(hit);
      if (m) {
        gfirst = min(gfirst, gb + (int)__builtin_ctzll(m));
        glast = gb + kWave - 1 - (int)__builtin_clzll(m);
      }
    }
    gfirst = __builtin_amdgcn_readfirstlane(gfirst);
    glast = __builtin_amdgcn_readfirstlane(glast);
    const int tb = t0 + ll * M;  // first target of this lane
    float acc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) acc[k] = 0.f;

    if (glast >= gfirst) {
      float sum[M], comp[M];
#pragma unroll
      for (int k = 0; k < M; ++k) sum[k] = comp[k] = 0.f;
      float fd = (float)(tb - (e_lo + gfirst * G + sl));  // target - source, exact
      int c = gfirst * G + sl;
      // one source of this stream against the lane's M targets
      auto pair_step = [&](const float4 q) {
        const float d0 = __builtin_fmaf(fd, dv, -q.z);
        const float tt0 = d0 * q.y;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const float t = (k == 0) ? tt0 : __builtin_fmaf((float)k, q.w, tt0);
          acc[k] = __builtin_fmaf(q.x, fexp2(-(t * t)), acc[k]);
        }
        fd -= (float)G;
      };
      auto fold = [&]() {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const float y = acc[k] - comp[k];
          const float tt = sum[k] + y;
          comp[k] = (tt - sum[k]) - y;
          sum[k] = tt;
          acc[k] = 0.f;
        }
      };
      // two records in flight: the LDS read of the next source overlaps the
      // arithmetic of the current one (rec is padded so the read past the
      // last group stays inside the array)
      float4 qa = rec[c];
      int g = gfirst, since = 0;
      for (; g + 1 <= glast; g += 2) {
        const float4 qb = rec[c + G];
        pair_step(qa);
        qa = rec[c + 2 * G];
        pair_step(qb);
        c += 2 * G;
        if (++since == KB / 2) {
          since = 0;
          fold();
        }
      }
      if (g <= glast) pair_step(qa);
      fold();
#pragma unroll
      for (int k = 0; k < M; ++k) acc[k] = stream_sum<S>(sum[k] - comp[k]);
    }
    // lanes sl = 0..M-1 of each stream group write one target each
    if (sl < M) {
      float o = acc[0];
#pragma unroll
      for (int k = 1; k < M; ++k) o = (sl == k) ? acc[k] : o;
      const int i = tb + sl;
      if (i < i_end) tau[off + i] = o;
    }
  }
}

// One work item (skewer, tile) per workgroup.
template <int S, int M, int TILE>
__global__ __launch_bounds__(kTauThreads) void tau_window_kernel(Batch b,
                                                                 const int2 *__restrict__ items,
                                                                 float *__restrict__ tau) {
  __shared__ float4 rec[kChunk + 2 * S];
  __shared__ float2 bnd[kChunk / S];
  tau_tile<S, M, TILE>(b, items[blockIdx.x], tau, rec, bnd);
}

// Persistent form: a grid sized to the resident workgroups takes items from a
// queue (the work list is sorted by estimated cost, largest first) until it is
// empty; every workgroup leaves the loop once the counter passes n_items.  A
// workgroup takes kQueueGrab consecutive items per atomic (the counter lives
// beyond the per-die L2 caches).  On the ragged 20000-skewer batch two items
// per grab took 1 % less time than four (the last grabs leave fewer
// workgroups idle) and eight 2 % more; one per grab measured the same as two.
constexpr int kQueueGrab = 2;
template <int S, int M, int TILE>
__global__ __launch_bounds__(kTauThreads) void tau_window_persistent_kernel(
    Batch b, const int2 *__restrict__ items, int n_items, unsigned int *queue,
    float *__restrict__ tau) {
  __shared__ float4 rec[kChunk + 2 * S];
  __shared__ float2 bnd[kChunk / S];
  __shared__ int next;
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and `next`
    if (threadIdx.x == 0) next = (int)atomicAdd(queue, (unsigned)kQueueGrab);
    __syncthreads();
    const int first = next;
    if (first >= n_items) break;
    const int last = min(first + kQueueGrab, n_items);
    for (int idx = first; idx < last; ++idx) {
      if (idx > first) __syncthreads();  // the previous item is done with LDS
      tau_tile<S, M, TILE>(b, items[idx], tau, rec, bnd);
    }
  }
}

__global__ void reset_queue_kernel(unsigned int *queue) { *queue = 0u; }

// ---------------------------------------------------------------------------
// Skewed windowed tile.  One source stream per wave: lane l owns the kSkewM
// consecutive targets i_l = t0 + 4l .. i_l + 3 of the wave's 256-target span
// and walks its own run of sources e = i_l - H .. i_l - H + NS - 1, where H
// and NS are wave-uniform.  The run therefore moves with the lane's targets:
// target minus source is the same integer H - s on every lane at step s, so
// no lane sees sources that only its neighbours need, and each lane finishes
// with its own sums (no cross-lane reduction).  H and NS come from a scan of
// the staged window bounds: H is the largest (lane start - source) and
// NS - H the largest (source - lane start) over the source/lane pairs whose
// window and targets meet.  Sources are staged in four planes by extended
// index mod 4, so the 64 lanes of a step read 64 consecutive float4 (no bank
// conflicts) and the four steps of an unrolled block use immediate offsets.
constexpr int kSkewM = 4;                  // targets per lane
constexpr int kSkewFold = 16;              // terms per block sum of a run
constexpr int kSkewPart = 8;               // block sums per partial sum
constexpr int kSkewMargin = 12;            // staged sources beyond the reach
constexpr int kSkewGroup = 4;              // sources per window-bounds group
// Target-minus-source offsets as exact floats, read from LDS four at a time
// (one broadcast read per block of four steps instead of a VALU decrement per
// step): entry k holds kFdTop - k.  A lane run covers offsets H4 .. H4 - NS + 1
// with H4 <= RH <= 476 and NS <= H4 + RH + M (M <= 8 targets per lane), plus
// one block read ahead.
constexpr int kSkewMaxRH = 476;  // staged margin limit of the windowed path
constexpr int kFdTop = 480;
constexpr int kFdN = 976;
static_assert(kFdTop >= kSkewMaxRH + 4 && kFdN >= kFdTop + kSkewMaxRH + 12 && kFdN % 4 == 0,
              "offset table covers every lane run");

template <int NWAVES, int M = kSkewM>
struct SkewShape {
  static_assert(M == 4 || M == 8, "a lane owns 4 or 8 targets");
  static constexpr int kLgM = M == 8 ? 3 : 2;
  static constexpr int kSpan = kWave * M;  // targets per wave
  static constexpr int kThreads = NWAVES * kWave;
  static constexpr int kTile = NWAVES * kSpan;
  // staged sources: tile + 2 RH with RH <= kMaxRH, so that four 4-wave
  // workgroups fit in the 160 KiB of LDS of a compute unit (tiles reaching
  // further take the full-sum path).  With 2048 targets the margin is smaller,
  // the window bounds are kept per 8 sources instead of 4, and the offsets
  // of a block of steps come from the VALU instead of a table in LDS.
  static constexpr int kMaxRH = M == 8 ? 200 : kSkewMaxRH;
  static constexpr int kChunkS =
      kTile + 2 * kMaxRH > kChunk ? kTile + 2 * kMaxRH : kChunk;
  static constexpr int kPlane = kChunkS / 4;
  static constexpr int kGroup = M == 8 ? 8 : kSkewGroup;  // sources per window-bounds group
  static constexpr int kGroups = kChunkS / kGroup;
  static constexpr bool kFdTable = M != 8;
  static constexpr int kFdEntries = kFdTable ? kFdN / 4 : 1;
  static_assert(kChunkS >= kChunk, "the full-sum path stages kChunk sources");
  static_assert((kChunkS + 4) * 16 + kGroups * 4 + kFdEntries * 16 + 16 <= 160 * 1024 / 4,
                "four workgroups per compute unit");
};

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m));
  return x;
}

// REC: the Gaussian recurrence across a lane's four targets.  With
// t_k = t_0 + k a (a = dv r), t_k^2 - t_(k-1)^2 = a (2 t_(k-1) + a), so
// E_k = exp2(-t_k^2) = E_(k-1) G_(k-1) with G_0 = exp2(-a (2 t_0 + a)) and
// G_k = G_(k-1) C, C = exp2(-2 a^2) per source: two exp2 per source and lane
// instead of four.  These records hold (w, a, v r, C), so that
// t_0 = (fd dv - v) r = fd a - v r is one FMA on the exact offset fd; a and
// v r are rounded once each, which adds about u (|fd a| + |v r|) to t_0 (on the
// 4096 x 4096 workload's fields, 1e-7 of tau at most).  The chain starts
// at the lane's first target; it is exact to rounding unless E_0 underflows
// while a later E_k matters, which needs a > 1.16 (|t_0| > 11.2 and
// |t_0 + 3a| < 7.75), so a tile with any source of a > kRecMaxA (unresolved
// lines) takes the direct form.  G_0 is clamped at 2^64, reached only where
// E_0 = 0 (t_0 < -32 for a <= 1), so that no product is 0 * inf.
// With 8 targets per lane the chain reaches 7a past its start: it is exact
// unless a > 0.49 (|t_0| > 11.2 and |t_0 + 7a| < 7.75).
constexpr float kRecMaxA = 1.0f;
constexpr float kRecMaxA8 = 0.45f;

template <int NWAVES, bool REC = false, int M = kSkewM>
__device__ __forceinline__ void tau_skew_tile(const Batch &b, const int2 item,
                                              float *__restrict__ tau, float4 *rec,
                                              int *gwin, const float4 *fdt) {
  using SH = SkewShape<NWAVES, M>;
  constexpr int TILE = SH::kTile, NT = SH::kThreads, PL = SH::kPlane;
  const int64_t s = item.x;
  const int i0 = item.y * TILE;
  const SkewerConst K = b.skc[s];
  const int64_t off = b.offsets[s];
  const int n = K.n;
  const int i_end = min(i0 + TILE, n);
  // staged margin on each side, a multiple of 4 so that lane runs start on a
  // plane-0 column
  const int RH = (K.reach + kSkewMargin + 3) & ~3;
  if (TILE + 2 * RH > SH::kChunkS || RH > SH::kMaxRH || 2 * RH + 8 > n) {
    // the window covers the box, or reaches beyond the staged margin
    for (int q = i0; q < i_end; q += NT) full_sum_tile<true>(b, K, off, q, tau, rec);
    return;
  }

  // ---- stage extended indices e_lo .. i_end + RH - 1 (position c = e - e_lo).
  // A thread issues its global reads in rounds of 8 ahead of the arithmetic
  // of the round.  The
  // window bounds of every group of 4 positions (lowest ceil(lo), highest
  // floor(hi)) meet in a DPP reduction over the 4 lanes that hold them.
  constexpr int SIT = 8;  // positions per thread per round of reads
  const int e_lo = i0 - RH;
  const int cnt = (i_end - i0) + 2 * RH;
  const float pivot = b.pivot, wk = b.window_k;
  bool bad = false;
  int unsafe = 0;  // REC: a source of a > kRecMaxA
  // CHAIN_LAYOUT: records (w, a, v r, C) for the recurrence, else (w, r, v, a)
  auto stage = [&](const bool chain_layout) {
    for (int c0 = 0; c0 < cnt; c0 += SIT * NT) {
      float dd[SIT], vv[SIT];
#pragma unroll
      for (int u = 0; u < SIT; ++u) {
        const int c = c0 + threadIdx.x + u * NT;
        dd[u] = 0.f;
        vv[u] = 0.f;
        if (c < cnt) {
          const int e = e_lo + c;  // -n <= e < 2n: RH <= n/2 and i_end <= n
          const int j = e < 0 ? e + n : (e >= n ? e - n : e);
          dd[u] = b.delta[off + j];
          vv[u] = b.vpec[off + j];
        }
      }
#pragma unroll
      for (int u = 0; u < SIT; ++u) {
        if (c0 + u * NT >= cnt) break;
        const int c = c0 + threadIdx.x + u * NT;
        bad |= (c < cnt) && bad_delta(dd[u]);
        const Src o = source_of(dd[u], K, pivot);
        float flo = 8191.f, fhi = -8192.f;  // no window: meets no target
        if (c < cnt) {
          if (o.w > 0.f) {
            const float cc = __builtin_fmaf(vv[u], K.inv_dv, (float)c);  // line centre
            const float h = wk * o.b * K.inv_dv;                         // half window
            flo = fminf(fmaxf(ceilf(cc - h), -8192.f), 8191.f);
            fhi = fminf(fmaxf(floorf(cc + h), -8192.f), 8191.f);
          }
          const float a = K.dv * o.r;
          if (chain_layout) {
            unsafe |= (o.w > 0.f) && !(a <= (M == 8 ? kRecMaxA8 : kRecMaxA));
            // (w, a = dv r, v r, C): t_0 = fd a - v r takes one FMA in the walk
            rec[(c & 3) * PL + (c >> 2)] = make_float4(o.w, a, vv[u] * o.r, fexp2(-2.f * a * a));
          } else {
            rec[(c & 3) * PL + (c >> 2)] = make_float4(o.w, o.r, vv[u], a);
          }
        }
        flo = stream_min<SH::kGroup>(flo);
        fhi = stream_max<SH::kGroup>(fhi);
        if ((threadIdx.x & (SH::kGroup - 1)) == 0 && c < cnt)
          gwin[c / SH::kGroup] =
              (int)(((uint32_t)(int)fhi & 0xFFFFu) | ((uint32_t)(int)flo << 16));
      }
    }
  };
  stage(REC);
  flag_bad_delta(b, bad);
  const bool chain = REC ? __syncthreads_or(unsafe) == 0 : false;
  if (!REC) __syncthreads();
  if (REC && !chain) {
    // the direct form keeps the exact offset d_0 = fd dv - v (one rounding)
    // and r: narrow lines, whose wings can carry a pixel's whole tau, would
    // otherwise take the rounding of v r at |v r| >> |t_0|.  The tile is
    // staged again with those records (Delta and v re-read, mostly from L2).
    stage(false);
    __syncthreads();
  }

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int t0 = i0 + wave * SH::kSpan;
  if (t0 >= i_end) return;
  const int T0r = t0 - e_lo;  // position of the wave's first target
  const int last_lane = min(kWave - 1, (i_end - 1 - t0) >> SH::kLgM);

  // ---- H and NS for this wave, from the groups whose windows meet its
  // targets: the group's first position bounds (lane start - source) from
  // above, its last position (source - lane start)
  int Hm = -(1 << 20), Em = -(1 << 20);
  {
    constexpr int G = SH::kGroup;
    const int g_beg = (T0r - RH) / G;
    const int g_end = min((cnt + G - 1) / G, (T0r + SH::kSpan + RH + G - 1) / G);
    for (int g = g_beg + lane; g < g_end; g += kWave) {
      const int x = gwin[g];
      const int fh = (int)(int16_t)(x & 0xFFFF) - T0r;  // floor(hi) - T0r
      const int fl = (x >> 16) - (M - 1) - T0r;
      const int lhi = min(fh >> SH::kLgM, last_lane);  // last lane whose targets the windows meet
      const int llo = max((fl + M - 1) >> SH::kLgM, 0);  // first such lane
      if (llo <= lhi) {
        Hm = max(Hm, T0r + M * lhi - G * g);
        Em = max(Em, G * g + G - 1 - T0r - M * llo);
      }
    }
    Hm = __builtin_amdgcn_readfirstlane(wave_max(Hm));
    Em = __builtin_amdgcn_readfirstlane(wave_max(Em));
  }
  const int H4 = min((Hm + 3) & ~3, RH);
  // a lane's sources reach RH past its last target: the run never needs more
  // than H4 + RH + M steps, which keeps every lane inside the staged range
  const int NS = min((H4 + Em + 1 + 3) & ~3, H4 + RH + M);
  const int i_l = t0 + M * lane;

  // sums of a lane's targets in three levels: acc over a block of kSkewFold
  // steps, part over up to kSkewPart blocks, sum over those (all terms are
  // positive: a relative error of at most (15 + 7 + NS / 128) u)
  float sum[M], part[M];
#pragma unroll
  for (int k = 0; k < M; ++k) sum[k] = part[k] = 0.f;
  if (Em >= -(1 << 19) && NS > 0) {
    const float dv = K.dv;
    float acc[M];
    // one source against the lane's kSkewM targets; fd is the exact target
    // minus source offset of the step; FIRST starts a new run
    auto pair_step = [&](const float4 q, const float fd, const bool first) {
      // records (w, r, v, a): the direct form of every shape
      const float tt0 = __builtin_fmaf(fd, dv, -q.z) * q.y;
      const float a = q.w;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const float t = (k == 0) ? tt0 : __builtin_fmaf((float)k, a, tt0);
        const float e = fexp2(-(t * t));
        acc[k] = first ? q.x * e : __builtin_fmaf(q.x, e, acc[k]);
      }
    };
    // one source against the lane's kSkewM targets by the recurrence
    auto pair_chain = [&](const float4 q, const float fd, const bool first) {
      const float tt0 = __builtin_fmaf(fd, q.y, -q.z);
      const float a = q.y;
      float E = fexp2(-(tt0 * tt0));
      float G = fexp2(fminf(-(__builtin_fmaf(2.f, tt0, a) * a), 64.f));
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if (k > 0) {
          E *= G;
          if (k + 1 < M) G *= q.w;
        }
        acc[k] = first ? q.x * E : __builtin_fmaf(q.x, E, acc[k]);
      }
    };
    // CH: the recurrence (decided per tile, so the whole walk takes one form
    // and its sums stay in the same registers from block to block)
    auto block = [&](auto ch, const float4 (&q)[5], const bool first) {
      if constexpr (decltype(ch)::value) {
        pair_chain(q[0], q[4].x, first);
        pair_chain(q[1], q[4].y, false);
        pair_chain(q[2], q[4].z, false);
        pair_chain(q[3], q[4].w, false);
        // the block's 8 exps, one per 7 (M = 4) or 18 (M = 8: the last ones
        // early, measured best) other VALU instructions
#pragma unroll
        for (int z = 0; z < 8; ++z) {
          __builtin_amdgcn_sched_group_barrier(0x400, 1, 0);            // one transcendental
          __builtin_amdgcn_sched_group_barrier(0x002, M == 8 ? 18 : 7, 0);  // VALU
        }
        return;
      } else {
        pair_step(q[0], q[4].x, first);
        pair_step(q[1], q[4].y, false);
        pair_step(q[2], q[4].z, false);
        pair_step(q[3], q[4].w, false);
        // the transcendental unit runs beside the other VALU work: the
        // block's 4 M exps are spread one per four other VALU instructions,
        // so that they do not queue behind one another
#pragma unroll
        for (int z = 0; z < 4 * M; ++z) {
          __builtin_amdgcn_sched_group_barrier(0x400, 1, 0);  // one transcendental
          __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // four VALU
        }
      }
    };
    int folds = 0;
    auto fold = [&]() {
#pragma unroll
      for (int k = 0; k < M; ++k) part[k] += acc[k];
      if (++folds == kSkewPart) {
        folds = 0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          sum[k] += part[k];
          part[k] = 0.f;
        }
      }
    };
    // column of the run's first source in every plane; a block is 4 steps
    // (one record from each plane), a run of kSkewFold steps is 4 blocks
    const float4 *p = rec + ((T0r - H4) >> 2) + lane * (M / 4);
    const float4 *pf = fdt + ((kFdTop - H4) >> 2);  // offsets H4 - 4 blk - (0..3)
    auto load = [&](float4 (&q)[5], const int blk) {
      q[0] = p[blk];
      q[1] = p[blk + PL];
      q[2] = p[blk + 2 * PL];
      q[3] = p[blk + 3 * PL];
      if constexpr (SH::kFdTable) {
        q[4] = pf[blk];
      } else {
        const float f = (float)(H4 - 4 * blk);
        q[4] = make_float4(f, f - 1.f, f - 2.f, f - 3.f);
      }
    };
    const int nblk = NS >> 2;
    static_assert(kSkewFold == 4 * 4, "the walk folds after four blocks of four steps");
    // the next block's records are read while this one is evaluated; the read
    // past the last block stays inside the staged array
    auto walk = [&](auto ch) {
      float4 qa[5], qb[5];
      load(qa, 0);
      int blk = 0;
      for (; blk + 4 <= nblk; blk += 4) {
        load(qb, blk + 1);
        block(ch, qa, true);
        load(qa, blk + 2);
        block(ch, qb, false);
        load(qb, blk + 3);
        block(ch, qa, false);
        load(qa, blk + 4);
        block(ch, qb, false);
        fold();
      }
      for (; blk < nblk; ++blk) {
        load(qb, blk + 1);
        block(ch, qa, true);
        fold();
#pragma unroll
        for (int k = 0; k < 5; ++k) qa[k] = qb[k];
      }
    };
    if constexpr (REC) {
      if (chain)
        walk(std::true_type{});
      else
        walk(std::false_type{});
    } else {
      walk(std::false_type{});
    }
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int i = i_l + k;
    if (i < i_end) tau[off + i] = sum[k] + part[k];
  }
}

__device__ __forceinline__ void fill_offset_table(float4 *fdt) {
  for (int k = threadIdx.x; k < kFdN / 4; k += blockDim.x) {
    const float t = (float)(kFdTop - 4 * k);
    fdt[k] = make_float4(t, t - 1.f, t - 2.f, t - 3.f);
  }
}

template <int NWAVES, bool REC, int M>
__global__ __launch_bounds__(NWAVES * kWave) void tau_skew_kernel(Batch b,
                                                                  const int2 *__restrict__ items,
                                                                  float *__restrict__ tau) {
  using SH = SkewShape<NWAVES, M>;
  __shared__ float4 rec[SH::kChunkS + 4];
  __shared__ int gwin[SH::kGroups];
  __shared__ float4 fdt[SH::kFdEntries];
  if (SH::kFdTable) fill_offset_table(fdt);  // published by the barrier after staging
  tau_skew_tile<NWAVES, REC, M>(b, items[blockIdx.x], tau, rec, gwin, fdt);
}

// 4-wave form: at most 128 VGPRs, so that four waves share a SIMD as in the
// grid form
template <int NWAVES, bool REC, int M>
__global__ __launch_bounds__(NWAVES * kWave)
__attribute__((amdgpu_waves_per_eu(NWAVES == 4 ? 4 : 3))) void tau_skew_persistent_kernel(
    Batch b, const int2 *__restrict__ items, int n_items, unsigned int *queue,
    float *__restrict__ tau) {
  using SH = SkewShape<NWAVES, M>;
  __shared__ float4 rec[SH::kChunkS + 4];
  __shared__ int gwin[SH::kGroups];
  __shared__ float4 fdt[SH::kFdEntries];
  __shared__ int next;
  if (SH::kFdTable) fill_offset_table(fdt);
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and `next`
    if (threadIdx.x == 0) next = (int)atomicAdd(queue, (unsigned)kQueueGrab);
    __syncthreads();
    const int first = next;
    if (first >= n_items) break;
    const int last = min(first + kQueueGrab, n_items);
    for (int idx = first; idx < last; ++idx) {
      if (idx > first) __syncthreads();  // the previous item is done with LDS
      tau_skew_tile<NWAVES, REC, M>(b, items[idx], tau, rec, gwin, fdt);
    }
  }
}

namespace {
struct VariantFns {
  const void *grid_fn;
  const void *pers_fn;
  int threads;
  void (*grid)(const Batch &, const int2 *, int64_t, float *, hipStream_t, hipEvent_t,
               hipEvent_t);
  void (*pers)(const Batch &, const int2 *, int64_t, unsigned int *, int, float *, hipStream_t);
};

template <int S, int M, int TILE>
VariantFns make_variant() {
  VariantFns v;
  v.grid_fn = reinterpret_cast<const void *>(&tau_window_kernel<S, M, TILE>);
  v.pers_fn = reinterpret_cast<const void *>(&tau_window_persistent_kernel<S, M, TILE>);
  v.threads = kTauThreads;
  v.grid = [](const Batch &b, const int2 *items, int64_t n, float *tau, hipStream_t st,
              hipEvent_t e0, hipEvent_t e1) {
    if (e0)
      hipExtLaunchKernelGGL((tau_window_kernel<S, M, TILE>), dim3((unsigned)n), dim3(kTauThreads),
                            0, st, e0, e1, 0, b, items, tau);
    else
      hipLaunchKernelGGL((tau_window_kernel<S, M, TILE>), dim3((unsigned)n), dim3(kTauThreads),
                         0, st, b, items, tau);
  };
  v.pers = [](const Batch &b, const int2 *items, int64_t n, unsigned int *queue, int grid,
              float *tau, hipStream_t st) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, st, queue);
    hipLaunchKernelGGL((tau_window_persistent_kernel<S, M, TILE>), dim3((unsigned)grid),
                       dim3(kTauThreads), 0, st, b, items, (int)n, queue, tau);
  };
  return v;
}

template <int NWAVES, bool REC = false, int M = kSkewM>
VariantFns make_skew_variant() {
  constexpr int NT = SkewShape<NWAVES, M>::kThreads;
  VariantFns v;
  v.grid_fn = reinterpret_cast<const void *>(&tau_skew_kernel<NWAVES, REC, M>);
  v.pers_fn = reinterpret_cast<const void *>(&tau_skew_persistent_kernel<NWAVES, REC, M>);
  v.threads = NT;
  v.grid = [](const Batch &b, const int2 *items, int64_t n, float *tau, hipStream_t st,
              hipEvent_t e0, hipEvent_t e1) {
    if (e0)
      hipExtLaunchKernelGGL((tau_skew_kernel<NWAVES, REC, M>), dim3((unsigned)n), dim3(NT), 0,
                            st, e0, e1, 0, b, items, tau);
    else
      hipLaunchKernelGGL((tau_skew_kernel<NWAVES, REC, M>), dim3((unsigned)n), dim3(NT), 0, st,
                         b, items, tau);
  };
  v.pers = [](const Batch &b, const int2 *items, int64_t n, unsigned int *queue, int grid,
              float *tau, hipStream_t st) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, st, queue);
    hipLaunchKernelGGL((tau_skew_persistent_kernel<NWAVES, REC, M>), dim3((unsigned)grid),
                       dim3(NT), 0, st, b, items, (int)n, queue, tau);
  };
  return v;
}

const VariantFns &variant_fns(int v) {
  static const VariantFns table[kNumTauVariants] = {
      make_skew_variant<4>(),
      make_skew_variant<2>(),
      make_variant<8, 4, 512>(),
      make_variant<8, 2, 512>(),
      make_skew_variant<4, true>(),     // the recurrence across a lane's targets (default)
      make_skew_variant<4, true, 8>(),  // the same over 8 targets per lane
  };
  return table[v];
}
}  // namespace

const TauVariant kTauVariants[kNumTauVariants] = {
    {1, kSkewM, SkewShape<4>::kTile}, {1, kSkewM, SkewShape<2>::kTile}, {8, 4, 512}, {8, 2, 512},
    {1, kSkewM, SkewShape<4>::kTile}, {1, 8, SkewShape<4, 8>::kTile}};

hipError_t launch_tau_window(const Batch &b, const int2 *items, int64_t n_items, float *tau,
                             hipStream_t st, int variant, int persistent_grid,
                             unsigned int *queue, hipEvent_t start, hipEvent_t stop) {
  if (n_items == 0) return hipSuccess;
  const VariantFns &f = variant_fns(variant);
  if (persistent_grid > 0)
    f.pers(b, items, n_items, queue, persistent_grid, tau, st);
  else
    f.grid(b, items, n_items, tau, st, start, stop);
  return hipGetLastError();
}

int tau_persistent_grid(int variant) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const VariantFns &f = variant_fns(variant);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f.pers_fn, f.threads, 0) !=
      hipSuccess)
    return 0;
  return std::max(1, cus * per_cu);
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
