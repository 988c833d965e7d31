// lyaf_adjoint.hip -- hand-written adjoint of the optical-depth sum (Greig,
// Bolton & Wyithe 2011, Section 2.3, eqs. 4-6), by the chain rule.
//
// For source j (weight w_j, Doppler parameter b_j, t = d_ij sqrt(log2 e) / b_j,
// so that exp(-x^2) = exp2(-t^2) with x = d_ij / b_j):
//   S0_j = w_j sum_i g_i E_ij,  S1_j = w_j sum_i g_i E_ij x_ij,
//   S2_j = w_j sum_i g_i E_ij x_ij^2,  Q_j = S2_j - 1.2 S0_j,
//   dL/dv_j = 2 S1_j / b_j,
//   dL/dDelta_j = [2 S0_j + (gamma-1) [Delta_j <= pivot] Q_j] / Delta_j,
//   dL/dT0 = sum_j Q_j / T0,   dL/dgamma = sum_j Q_j ln D_j.
// The 1.2 is the temperature exponent of w (n_HI ~ T^-0.7 over b ~ T^0.5).
//
// One workgroup per 256-source pass; the target gradients g_i within reach are
// staged in LDS.  Each lane owns one source and walks its own run of targets,
// four per step, shifted with its source: the run of lane l starts at j_l - H
// and has NS targets, H and NS uniform over the wave (from the lanes' window
// bounds), so target minus source is the same on every lane and the four
// targets of a step share t_k = t_0 + k a (a = dv r).  Short or wide skewers
// sum over every target with the minimal image chosen per pair.  The three
// per-source sums are FP32 blocks of 16 terms folded with Kahan compensation
// (S1 is a signed sum that cancels across the line centre), Q_j is formed in
// FP64 from them, and the per-skewer T0/gamma terms are summed in FP64 per
// workgroup and then per skewer in a fixed order.
#include <math.h>

#include "lyaf_internal.h"

namespace lyaf {

__device__ __forceinline__ float aexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float alog2(float x) { return __builtin_amdgcn_logf(x); }

constexpr int kAdjThreads = 256;
constexpr int kAdjTile = 256;  // sources per pass of the workgroup (one per thread)
constexpr int kAdjMargin = 12; // staged targets beyond the reach

// Compensated sum of FP32 blocks: sum + comp carries the running total.
struct KahanSum {
  float sum = 0.f, comp = 0.f;
  __device__ __forceinline__ void add(const float blk) {
    const float y = blk - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  __device__ __forceinline__ float value() const { return sum - comp; }
};

__device__ __forceinline__ int adj_wave_max(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m));
  return x;
}
static_assert(kTauTile % kAdjTile == 0, "work items hold whole adjoint passes");

// One pass: sources j0 .. j0+255 of skewer s (one per thread).  Adds this
// thread's Q_j and Q_j ln D_j to q_T0 and q_gam.
__device__ void adjoint_pass(const Batch &b, const SkewerConst &K, int64_t off, int j0,
                             const float *__restrict__ g, float *__restrict__ gdelta,
                             float *__restrict__ gvpec, float *gl, double &q_T0,
                             double &q_gam) {
  const int n = K.n;
  const int R = K.reach;
  const int j = j0 + (int)threadIdx.x;
  const bool valid = j < n;

  // this lane's source
  float delta = 0.f, v = 0.f, w = 0.f, r = K.R, bj = 0.f, l2D = 0.f;
  if (valid) {
    delta = b.delta[off + j];
    v = b.vpec[off + j];
    if (delta > 0.f) {
      const float D = fmaxf(fminf(delta, b.pivot), 1e-30f);
      l2D = alog2(D);
      const float x = K.gm1 * l2D;
      w = K.W * delta * delta * aexp2(kTempExpW * x);
      r = K.R * aexp2(kTempExpR * x);
      bj = K.B * aexp2(0.5f * x);
    }
  }
  // an invalid density sets the sticky domain bit (the reach pass may not
  // have read Delta)
  if (__any(valid && (!(delta >= 0.f) || !isfinite(delta))) && (threadIdx.x & 63) == 0)
    atomicOr(b.status, LYAF_STATUS_DOMAIN);
  const float dv = K.dv;
  // sums of g E, g E t, g E t^2: blocks of 16 terms folded into Kahan sums
  float S0 = 0.f, S1 = 0.f, S2 = 0.f;
  KahanSum K0, K1, K2;
  auto fold = [&]() {
    K0.add(S0);
    K1.add(S1);
    K2.add(S2);
    S0 = S1 = S2 = 0.f;
  };

  // staged margin beyond the reach (window bounds are rounded outwards)
  const int RH = (R + kAdjMargin + 3) & ~3;
  const int j_end = min(j0 + kAdjTile, n);
  const int e_lo = j0 - RH;
  const int cnt = (j_end - j0) + 2 * RH;
  __syncthreads();  // gl is reused across passes
  if (kAdjTile + 2 * RH + 8 <= kChunk && 2 * RH + 8 <= n) {
    // windowed: targets e_lo .. e_lo + cnt - 1 (extended, periodic)
    for (int c = threadIdx.x; c < cnt; c += kAdjThreads) {
      const int e = e_lo + c;  // -n <= e < 2n
      const int i = e < 0 ? e + n : (e >= n ? e - n : e);
      gl[c] = g[off + i];
    }
    __syncthreads();
    // this lane's window in targets: j - Hl .. j + El
    int Hl = -(1 << 20), El = -(1 << 20);
    if (w > 0.f) {
      const float cc = __builtin_fmaf(v, K.inv_dv, (float)(j - j0));  // line centre
      const float h = b.window_k * bj * K.inv_dv;
      const float lo = fminf(fmaxf(ceilf(cc - h), -8192.f), 8191.f);
      const float hi = fminf(fmaxf(floorf(cc + h), -8192.f), 8191.f);
      Hl = (j - j0) - (int)lo;
      El = (int)hi - (j - j0);
    }
    const int H = min(__builtin_amdgcn_readfirstlane(adj_wave_max(Hl)), RH);
    const int E = __builtin_amdgcn_readfirstlane(adj_wave_max(El));
    if (E >= -(1 << 19)) {
      // NS <= H + RH - 8 keeps every read inside the staged targets
      const int NS = min((H + E + 1 + 3) & ~3, H + RH - 8);
      const float *gp = gl + (j - j0) + RH - H;  // run start of this lane
      const float a = dv * r;
      float fd = (float)(-H);  // target - source at the step's first target, exact
      for (int st = 0; st < NS; st += 4) {
        const float gi[4] = {gp[st], gp[st + 1], gp[st + 2], gp[st + 3]};
        const float t0 = __builtin_fmaf(fd, dv, -v) * r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float t = (k == 0) ? t0 : __builtin_fmaf((float)k, a, t0);
          const float tt = t * t;
          const float gE = gi[k] * aexp2(-tt);
          S0 += gE;
          S1 = __builtin_fmaf(gE, t, S1);
          S2 = __builtin_fmaf(gE, tt, S2);
        }
        fd += 4.f;
        if ((st & 12) == 12) fold();  // every 4 steps (16 terms); st is wave-uniform
      }
    }
  } else {
    // every target, minimal image per pair
    const float nf = (float)n;
    const float invV = 1.f / (nf * dv);
    for (int c0 = 0; c0 < n; c0 += kChunk) {
      const int cn = min(kChunk, n - c0);
      __syncthreads();
      for (int c = threadIdx.x; c < cn; c += kAdjThreads) gl[c] = g[off + c0 + c];
      __syncthreads();
      float fd = (float)(c0 - j);
      for (int c = 0; c < cn; ++c) {
        const float gi = gl[c];
        const float d0 = __builtin_fmaf(fd, dv, -v);
        const float img = floorf(__builtin_fmaf(d0, invV, 0.5f));
        const float d = __builtin_fmaf(__builtin_fmaf(img, -nf, fd), dv, -v);
        const float t = d * r;
        const float gE = gi * aexp2(-(t * t));
        const float gEt = gE * t;
        S0 += gE;
        S1 += gEt;
        S2 = __builtin_fmaf(gEt, t, S2);
        fd += 1.f;
        if ((c & 15) == 15) fold();
      }
      fold();
    }
  }
  fold();

  // per-source outputs (t = x sqrt(log2 e): x = t / sqrt(log2 e))
  if (valid) {
    float gd = 0.f, gv = 0.f;
    if (w > 0.f) {
      const float inv_s = (float)(1.0 / kSqrtLog2e);
      const float s0 = w * K0.value();
      const float s1 = w * K1.value() * inv_s;
      // Q = S2 - 1.2 S0 cancels where x^2 ~ 1.2: formed in FP64
      const double Q =
          (double)w * ((double)K2.value() * (1.0 / kLog2e) - 1.2 * (double)K0.value());
      gv = 2.f * s1 / bj;
      const float below = (delta <= b.pivot) ? 1.f : 0.f;
      gd = (float)((2.0 * (double)s0 + (double)K.gm1 * below * Q) / (double)delta);
      q_T0 += Q;
      q_gam += Q * ((double)l2D * kLn2);  // Q ln D
    }
    gdelta[off + j] = gd;
    gvpec[off + j] = gv;
  }
}

__global__ __launch_bounds__(kAdjThreads) void tau_adjoint_kernel(
    Batch b, const int2 *__restrict__ items, const float *__restrict__ g,
    float *__restrict__ gdelta, float *__restrict__ gvpec, double *__restrict__ gpart) {
  __shared__ float gl[kChunk];
  __shared__ double shd[8];
  const int2 item = items[blockIdx.x];
  const int64_t s = item.x;
  const SkewerConst K = b.skc[s];
  const int64_t off = b.offsets[s];
  double q_T0 = 0.0, q_gam = 0.0;
  for (int p = 0; p < kTauTile; p += kAdjTile) {
    const int j0 = item.y * kTauTile + p;
    if (j0 >= K.n) break;
    adjoint_pass(b, K, off, j0, g, gdelta, gvpec, gl, q_T0, q_gam);
  }
  // FP64 workgroup sums of Q (for dL/dT0 after division by T0) and Q ln D
  double a0 = q_T0, a1 = q_gam;
  for (int m = 32; m >= 1; m >>= 1) {
    a0 += __shfl_xor(a0, m);
    a1 += __shfl_xor(a1, m);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    shd[wv] = a0;
    shd[4 + wv] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    gpart[2 * (int64_t)blockIdx.x + 0] = (shd[0] + shd[1]) + (shd[2] + shd[3]);
    gpart[2 * (int64_t)blockIdx.x + 1] = (shd[4] + shd[5]) + (shd[6] + shd[7]);
  }
}

// Per-skewer fixed-order sum of the workgroup partials.  Items of skewer s are
// item_base[s] .. item_base[s+1]-1.
__global__ void adjoint_skewer_sum_kernel(const double *__restrict__ gpart,
                                          const int64_t *__restrict__ item_base,
                                          const float *__restrict__ T0, int64_t S,
                                          double *__restrict__ gT0,
                                          double *__restrict__ ggamma) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double q = 0.0, ql = 0.0;
  for (int64_t k = item_base[s]; k < item_base[s + 1]; ++k) {
    q += gpart[2 * k + 0];
    ql += gpart[2 * k + 1];
  }
  if (gT0) gT0[s] = q / (double)T0[s];
  if (ggamma) ggamma[s] = ql;
}

hipError_t launch_tau_adjoint(const Batch &b, const int2 *items, int64_t n_items,
                              const int64_t *item_base_dev, const float *g, float *gdelta,
                              float *gvpec, double *gT0, double *ggamma, double *gpart,
                              hipStream_t st) {
  if (n_items > 0)
    hipLaunchKernelGGL(tau_adjoint_kernel, dim3((unsigned)n_items), dim3(kAdjThreads), 0, st, b,
                       items, g, gdelta, gvpec, gpart);
  if (b.n_skewers > 0 && (gT0 || ggamma))
    hipLaunchKernelGGL(adjoint_skewer_sum_kernel, dim3((unsigned)((b.n_skewers + 255) / 256)),
                       dim3(256), 0, st, gpart, item_base_dev, b.T0, b.n_skewers, gT0, ggamma);
  return hipGetLastError();
}

}  // namespace lyaf
