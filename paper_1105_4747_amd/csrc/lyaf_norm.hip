// lyaf_norm.hip -- mean-flux renormalisation of Section 2.3 (Greig, Bolton &
// Wyithe 2011): find A with (1/P) sum_p exp(-A tau_p) = target_F over all
// pixels, then tau' = A tau and F = exp(-tau'); plus its backward pass.
//
// The root-find runs on the device without host synchronisation, as a short
// fixed sequence of kernels (each kernel boundary costs a few microseconds,
// so there are few):
//   norm_gather    8192 pixels spread evenly over the batch (all of them if
//                  fewer) into a contiguous buffer;
//   norm_sample    one workgroup keeps the sample in registers and iterates
//                  to convergence on it, starting from the Jensen
//                  lower bound A0 = -ln F / <tau> (g(A0) >= 0 for the convex,
//                  decreasing g(A) = <exp(-A tau)> - F); FP32 exponentials,
//                  FP64 sums.  The sample's root is within a few 1e-2 of the
//                  batch's (the sampling error of g is a few 1e-3).
//   norm_pass x3   S_k = sum tau^k exp(-A tau) over every pixel, in FP64 per
//                  workgroup, with the counts of zero and invalid values.
//                  After a settled sample the passes are exact from the
//                  first: FP64 exponentials (to 2e-13), k = 0 .. 5.  Each
//                  pass begins with every workgroup summing the previous
//                  pass's partials in the same fixed order and taking the
//                  same step: the root of the degree-5 Taylor series of g
//                  about A (the scaled moments M_k = A^k S_k / P are its
//                  coefficients up to sign and k!), accepted at once when it
//                  is below 0.1 of A and the degree-4 series' root agrees
//                  with it to 1e-8; otherwise a safeguarded Halley step
//                  (Newton, then bisection, as fallbacks) inside the bracket,
//                  accepted below 1e-5 of A.  A sample without a settled root
//                  starts the passes with FP32 exponentials and k = 0 .. 2
//                  until a Halley step is below 3e-2 of A.  A kernel
//                  boundary, not a device-scope fence, publishes the
//                  partials: on a multi-XCD part a fence per workgroup
//                  writes back and invalidates L2 and serialises the pass.
//   norm_finalise  the last step, then tau' = A tau and F = exp(-tau').
// From a sample root a few 1e-2 off, the degree-5 series' root is within
// ~1e-11 of the batch's root and the degree-4 one within ~1e-9 (lognormal-
// field tau), so one exact pass usually suffices: the second pass takes the
// step and returns, and the third (a reserve for the Halley iteration) and the
// finalisation find nothing left to do.  Results are bitwise reproducible.
#include <math.h>

#include <mutex>

#include "lyaf_internal.h"

namespace lyaf {

// exp(-x) for x >= 0 in FP64: Cody-Waite reduction x = k ln2 + r with
// |r| <= ln2/2 (ln2 split into a 32-bit head and a tail so k*ln2_hi is exact),
// then the Taylor series of exp(-r) to degree 13 (truncation below 1e-17).
// Full-rate FP64 arithmetic only: adding 1.5 2^52 inside one FMA rounds
// x log2 e to the integer k, which the low word of that sum holds, and 2^-k
// is built from its exponent bits.  Below 2^-1021 (x > 708) the result is 0.
__device__ __forceinline__ double exp_neg(double x) {
  if (!(x <= 708.0)) return 0.0;
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double shifter = 6755399441055744.0;  // 1.5 2^52
  const double t = fma(x, kLog2e, shifter);
  const double k = t - shifter;
  const int ki = __double2loint(t);
  double r = fma(-k, ln2_hi, x);
  r = fma(-k, ln2_lo, r);
  const double y = -r;
  double p = 1.0 / 6227020800.0;          // 1/13!
  p = fma(p, y, 1.0 / 479001600.0);       // 1/12!
  p = fma(p, y, 1.0 / 39916800.0);
  p = fma(p, y, 1.0 / 3628800.0);
  p = fma(p, y, 1.0 / 362880.0);
  p = fma(p, y, 1.0 / 40320.0);
  p = fma(p, y, 1.0 / 5040.0);
  p = fma(p, y, 1.0 / 720.0);
  p = fma(p, y, 1.0 / 120.0);
  p = fma(p, y, 1.0 / 24.0);
  p = fma(p, y, 1.0 / 6.0);
  p = fma(p, y, 0.5);
  p = fma(p, y, 1.0);
  p = fma(p, y, 1.0);
  return p * __hiloint2double((1023 - ki) << 20, 0);  // p 2^-k
}

// exp(-x) for x >= 0 to 2e-13 relative (the moments of the exact phase need
// ~1e-10): x = (n/256) ln2 + r with |r| <= ln2/512, 2^(-n/256) =
// 2^-(n >> 8) tab[n & 255] with tab[j] = 2^(-j/256), and exp(-r) by its Taylor
// series to degree 3 (truncation below 1.5e-13).  Branch-free: x is clamped at
// 745 (NaN too) and the exponent field of 2^-(n >> 8) at zero, so the result
// is 0 beyond x ~ 709 and below 2^-1021 from 708 on.
__device__ __forceinline__ double exp_neg_tab(double x, const double *tab) {
  const double xc = fmin(x, 745.0);
  const double shifter = 6755399441055744.0;  // 1.5 2^52
  const double t = fma(xc, 256.0 * kLog2e, shifter);
  const double n = t - shifter;
  const int ni = __double2loint(t);
  const double r = fma(-n, kLn2 / 256.0, xc);
  double p = 1.0 / 6.0;
  p = fma(p, -r, 0.5);
  p = fma(p, -r, 1.0);
  p = fma(p, -r, 1.0);
  const int ex = max(1023 - (ni >> 8), 0);
  return tab[ni & 255] * p * __hiloint2double(ex << 20, 0);
}

// Sum of N values over a workgroup of NW waves (fixed order), in every
// thread.  For many values thread q < N adds up quantity q's NW wave sums, so
// that no thread holds all N NW of them in registers at once (an extra
// barrier); few are added up by every thread.  sh holds N (NW + 1) doubles.
constexpr int block_sum_lds(int N, int NW) { return N * (NW + 1); }
template <int N, int NW>
__device__ __forceinline__ void block_sum(double (&v)[N], double *sh) {
#pragma unroll
  for (int q = 0; q < N; ++q)
    for (int m = 32; m >= 1; m >>= 1) v[q] += __shfl_xor(v[q], m);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) sh[q * NW + w] = v[q];
  __syncthreads();
  if constexpr (N * NW <= 16) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double t = sh[q * NW];
#pragma unroll
      for (int k = 1; k < NW; ++k) t += sh[q * NW + k];
      v[q] = t;
    }
  } else {
    if (threadIdx.x < N) {
      const double *r = sh + threadIdx.x * NW;
      double t = r[0];
#pragma unroll
      for (int k = 1; k < NW; ++k) t += r[k];
      sh[N * NW + threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = sh[N * NW + q];
  }
  __syncthreads();
}

// Fixed-order reduction of NQ partial quantities written per workgroup.
template <int NQ, int NW>
__device__ __forceinline__ void reduce_partials(const double *partials, int nblocks,
                                                double (&tot)[NQ], double *sh) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) tot[q] = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += blockDim.x)
#pragma unroll
    for (int q = 0; q < NQ; ++q) tot[q] += partials[k * kPartStride + q];
  block_sum<NQ, NW>(tot, sh);
}

constexpr int kNormThreads = 256;  // backward kernels and finalise
constexpr int kNormWaves = kNormThreads / kWave;
constexpr int kPassThreads = 512;  // full root-find passes
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kPassBatch = 4;    // float4 reads in flight per thread in a pass
// per-workgroup partials of a pass: S_0 .. S_5, #(tau = 0), #(invalid tau)
constexpr int kNormQ = 8;
constexpr int kQZero = 6, kQBad = 7;
static_assert(kNormQ <= kPartStride, "a workgroup's partials fit its slot");
constexpr int kSampleThreads = 256;
constexpr int kSampleWaves = kSampleThreads / kWave;
constexpr int kGatherThreads = 256;
constexpr int kSampleIters = 32;
// the sample iteration stops at this step: its root is only ~1e-2 from the
// batch's, which the first full pass's series step corrects
constexpr double kSampleTol = 1e-3;
constexpr double kFP32Accept = 3e-2;
// An exact-phase step from the degree-5 Taylor model of g is accepted at once
// when it is at most kTaylorMaxStep of A and the degree-4 model's root agrees
// with it to kTaylorAgree (the next term of the series, which bounds the
// degree-5 root's error, is then smaller by another factor of the step).
constexpr double kTaylorMaxStep = 0.1;
constexpr double kTaylorAgree = 1e-8;

// One safeguarded Halley step for g, g' = g1, g'' = g2 at s.A, narrowing the
// bracket; sets s.A and s.step = |A_new - A_old| / A_new.
__device__ __forceinline__ void halley(NormState &s, double g, double g1, double g2) {
  double An = s.A;
  if (g != 0.0) {
    if (g > 0.0) s.lo = s.A; else s.hi = s.A;
    const double den = 2.0 * g1 * g1 - g * g2;
    const double hal = (den != 0.0) ? s.A - 2.0 * g * g1 / den : NAN;
    const double newton = (g1 < 0.0) ? s.A - g / g1 : NAN;
    if (hal > s.lo && hal < s.hi) An = hal;
    else if (newton > s.lo && newton < s.hi) An = newton;
    else if (isfinite(s.hi)) An = 0.5 * (s.lo + s.hi);
    else An = 2.0 * s.A;
  }
  s.step = (g == 0.0) ? 0.0 : fabs(An - s.A) / An;
  s.A = An;
  s.iter += 1;
}

// The sample: pixel floor(k P / N) for k < N = min(P, kSampleN), gathered by
// many workgroups into a contiguous buffer (one workgroup pulling thousands of
// scattered cache lines alone would take tens of microseconds).
__global__ __launch_bounds__(kGatherThreads) void norm_gather_kernel(
    const float *__restrict__ tau, int64_t P, float *__restrict__ sample) {
  const int64_t N = P < kSampleN ? P : kSampleN;
  const int64_t k = (int64_t)blockIdx.x * kGatherThreads + threadIdx.x;
  if (k < N) sample[k] = tau[(k * P) / N];
}

// Root of the sample's g: one workgroup of four waves, the sample in LDS.
// Leaves the state for the full passes (FP32 phase, open bracket, no moments
// yet).
__global__ __launch_bounds__(kSampleThreads) void norm_sample_kernel(
    const float *__restrict__ sample, int64_t P, double target, NormState *st_out) {
  __shared__ double sh[block_sum_lds(3, kSampleWaves)];
  __shared__ float4 xs[kSampleN / 4];
  const int64_t N = P < kSampleN ? P : kSampleN;
  double v[3] = {0.0, 0.0, 0.0};  // sum tau, #zeros, #invalid over the sample
  constexpr int R = kSampleN / 4 / kSampleThreads;  // float4 per thread
  float4 q[R];
#pragma unroll
  for (int j = 0; j < R; ++j)  // every read in flight at once
    q[j] = reinterpret_cast<const float4 *>(sample)[threadIdx.x + j * kSampleThreads];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int k4 = threadIdx.x + j * kSampleThreads;
    float t[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bool in = 4 * (int64_t)k4 + c < N;  // slots past N hold tau = 0
      const bool bad = in && (!(t[c] >= 0.f) || !isfinite(t[c]));
      t[c] = (in && !bad) ? t[c] : 0.f;
      v[0] += (double)t[c];
      v[1] += (in && !bad && t[c] == 0.f) ? 1.0 : 0.0;
      v[2] += bad ? 1.0 : 0.0;
    }
    xs[k4] = make_float4(t[0], t[1], t[2], t[3]);
  }
  block_sum<3, kSampleWaves>(v, sh);  // its barriers publish xs
  NormState s;
  s.P = (double)P;
  s.Ps = (double)N;
  s.target = target;
  s.step = INFINITY;
  s.iter = 0;
  s.done = 0;
  s.status = 0;
  s.phase = kNormPhaseFP32;
  s.pending = 1;
  s.buf = 0;
  s.nparts = 0;
  s.lo = 0.0;
  s.hi = INFINITY;
  const double mean = v[0] / s.Ps;
  s.A = (mean > 0.0) ? -log(target) / mean : 1.0;
  // iterate only if the sample is valid and has a root; otherwise the full
  // passes start from A0 and settle the status
  if (v[2] == 0.0 && v[1] / s.Ps < target && mean > 0.0) {
    const double pad = (double)(kSampleN - N);
    for (int it = 0; it < kSampleIters; ++it) {
      const float Al = (float)(s.A * kLog2e);
      float e0 = 0.f, e1 = 0.f, e2 = 0.f;
      for (int k4 = threadIdx.x; k4 < kSampleN / 4; k4 += kSampleThreads) {
        const float4 q = xs[k4];
        const float t[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float e = __builtin_amdgcn_exp2f(-(Al * t[c]));
          e0 += e;
          e1 = __builtin_fmaf(t[c], e, e1);
          e2 = __builtin_fmaf(t[c] * t[c], e, e2);
        }
      }
      double m[3] = {(double)e0, (double)e1, (double)e2};
      block_sum<3, kSampleWaves>(m, sh);
      const double g = (m[0] - pad) / s.Ps - target;
      halley(s, g, -m[1] / s.Ps, m[2] / s.Ps);
      if (s.step <= kSampleTol) break;
    }
    // a settled sample root is close enough for the exact phase's series step
    if (s.step <= kSampleTol) s.phase = kNormPhaseExact;
  }
  s.lo = 0.0;
  s.hi = INFINITY;
  if (threadIdx.x == 0) *st_out = s;
}

// Root d of the degree-D Taylor model of g about A in the relative step
// (A_new = A (1 + d)): sum_{n <= D} (-1)^n M_n d^n / n! = target, with the
// scaled moments M_n = <(A tau)^n exp(-A tau)>, by Newton's method from d0;
// NaN if it does not settle.
template <int D>
__device__ double taylor_root(const double (&M)[6], double target, double d0) {
  double c[D + 1];
  double f = 1.0;  // n!
#pragma unroll
  for (int n = 0; n <= D; ++n) {
    if (n > 0) f *= (double)n;
    c[n] = ((n & 1) ? -M[n] : M[n]) / f;
  }
  c[0] -= target;
  double d = d0;
#pragma unroll 1
  for (int it = 0; it < 40; ++it) {
    double p = c[D], dp = (double)D * c[D];
#pragma unroll
    for (int n = D - 1; n >= 1; --n) {
      p = fma(p, d, c[n]);
      dp = fma(dp, d, (double)n * c[n]);
    }
    p = fma(p, d, c[0]);
    const double dn = d - p / dp;
    if (!isfinite(dn)) return NAN;
    if (fabs(dn - d) <= 4e-16 * fabs(dn) + 1e-300) return dn;  // settled to rounding
    d = dn;
  }
  return NAN;
}

// One step from full-pass moments (with the domain and root-existence checks
// on the counts), and the phase change.
__device__ NormState norm_step(NormState s, const double (&tot)[kNormQ]) {
  if (tot[kQBad] > 0.0) {
    s.done = 1;
    s.status |= LYAF_STATUS_DOMAIN;
    return s;
  }
  if (!(tot[kQZero] / s.P < s.target)) {
    s.done = 1;
    s.status |= LYAF_STATUS_NOROOT;
    return s;
  }
  if (s.phase == kNormPhaseExact) {
    // the series of g about A: accepted at once when its degree-4 and
    // degree-5 roots agree and the step is small
    double M[6];
    double An = 1.0;  // A^n
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      M[n] = An * tot[n] / s.P;
      An *= s.A;
    }
    const double den = 2.0 * M[1] * M[1] - (M[0] - s.target) * M[2];
    const double d0 = (den > 0.0) ? 2.0 * (M[0] - s.target) * M[1] / den : 0.0;  // Halley
    const double d5 = taylor_root<5>(M, s.target, d0);
    const double d4 = taylor_root<4>(M, s.target, d5);
    if (fabs(d5) <= kTaylorMaxStep && fabs(d5 - d4) <= kTaylorAgree) {
      const double Anew = s.A * (1.0 + d5);
      s.step = fabs(Anew - s.A) / Anew;
      s.A = Anew;
      s.iter += 1;
      s.done = 1;
      return s;
    }
  }
  halley(s, tot[0] / s.P - s.target, -tot[1] / s.P, tot[2] / s.P);
  // a step below kNormAcceptStep of A leaves an iterate within ~K 1e-15 of
  // the root, accepted without another pass.  The FP32 phase hands over with
  // an open bracket: the signs of g it saw carry the FP32 error.
  if (s.phase == kNormPhaseExact) {
    if (s.step <= kNormAcceptStep) s.done = 1;
  } else if (s.step <= kFP32Accept) {
    s.phase = kNormPhaseExact;
    s.lo = 0.0;
    s.hi = INFINITY;
  }
  return s;
}

// A full pass.  Every workgroup reads the state the previous kernel left,
// sums the previous pass's partials in the same fixed order and takes the
// same step; workgroup 0 records the result.  Then S0..S2 at the new A (FP32
// or FP64 exponentials by phase) and the counts, per workgroup.
__global__ __launch_bounds__(kPassThreads) void norm_pass_kernel(
    const float *__restrict__ tau, int64_t P, double *partials, const NormState *st_prev,
    NormState *st_out, uint32_t *status) {
  __shared__ double sh[block_sum_lds(kNormQ, kPassWaves)];
  __shared__ NormState shs;
  if (threadIdx.x == 0) shs = *st_prev;
  __syncthreads();
  NormState s = shs;
  if (s.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *st_out = s;
    return;
  }
  if (!s.pending) {
    double tot[kNormQ];
    reduce_partials<kNormQ, kPassWaves>(partials + s.buf * kPartStride * kMaxPartialBlocks,
                                        s.nparts, tot, sh);
    if (threadIdx.x == 0) shs = norm_step(s, tot);
    __syncthreads();
    s = shs;
    if (s.done) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        *st_out = s;
        if (s.status) atomicOr(status, (uint32_t)s.status);
      }
      return;
    }
  }
  const int out_buf = 1 - s.buf;
  const bool aligned = (reinterpret_cast<uintptr_t>(tau) & 15) == 0;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P4 = P >> 2;  // whole groups of four pixels; the tail below
  double m[kNormQ] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int nz = 0, nbad = 0;
  auto counts = [&](float t) {
    nz += (t == 0.f);
    nbad += (!(t >= 0.f) || !isfinite(t));
  };
  auto group = [&](int64_t i) {  // pixels 4i .. 4i+3
    if (aligned) return reinterpret_cast<const float4 *>(tau)[i];
    return make_float4(tau[4 * i], tau[4 * i + 1], tau[4 * i + 2], tau[4 * i + 3]);
  };
  const int64_t tail = P - 4 * P4;  // 0..3 pixels, one per thread of the first threads
  // this thread's groups gtid, gtid + nthr, ...: kPassBatch reads issued
  // before any is used, so that their latency overlaps the arithmetic of the
  // others, then the rest one at a time
  auto strided = [&](auto &&use) {
    int64_t i = gtid;
    for (; i + (kPassBatch - 1) * nthr < P4; i += kPassBatch * nthr) {
      float4 t[kPassBatch];
#pragma unroll
      for (int b = 0; b < kPassBatch; ++b) t[b] = group(i + b * nthr);
#pragma unroll
      for (int b = 0; b < kPassBatch; ++b) use(t[b]);
    }
    for (; i < P4; i += nthr) use(group(i));
  };
  if (s.phase == kNormPhaseFP32) {
    const float Al = (float)(s.A * kLog2e);
    float e0 = 0.f, e1 = 0.f, e2 = 0.f;
    auto px = [&](float t) {
      const float e = __builtin_amdgcn_exp2f(-(Al * t));
      e0 += e;
      e1 = __builtin_fmaf(t, e, e1);
      e2 = __builtin_fmaf(t * t, e, e2);
      counts(t);
    };
    auto quad = [&](const float4 t) {
      px(t.x);
      px(t.y);
      px(t.z);
      px(t.w);
      m[0] += (double)e0;  // FP32 sums of four terms, then FP64
      m[1] += (double)e1;
      m[2] += (double)e2;
      e0 = e1 = e2 = 0.f;
    };
    strided(quad);
    if (gtid < tail) {
      px(tau[4 * P4 + gtid]);
      m[0] += (double)e0;
      m[1] += (double)e1;
      m[2] += (double)e2;
    }
  } else {
    __shared__ double tab[256];  // 2^(-j/256)
    static_assert(kPassThreads >= 256, "one table entry per thread");
    if (threadIdx.x < 256) tab[threadIdx.x] = exp_neg(threadIdx.x * (kLn2 / 256.0));
    __syncthreads();
    const double A = s.A;
    auto px = [&](float tf, double (&acc)[6]) {  // tau^n exp(-A tau), n = 0 .. 5
      const double t = (double)tf;
      double te = exp_neg_tab(A * t, tab);
      acc[0] += te;
#pragma unroll
      for (int n = 1; n < 6; ++n) {
        te *= t;
        acc[n] += te;
      }
      counts(tf);
    };
    // two sets of sums, alternate pixels (shorter dependency chains)
    double m1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, m2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    strided([&](const float4 t) {
      px(t.x, m1);
      px(t.y, m2);
      px(t.z, m1);
      px(t.w, m2);
    });
    if (gtid < tail) px(tau[4 * P4 + gtid], m1);
#pragma unroll
    for (int n = 0; n < 6; ++n) m[n] = m1[n] + m2[n];
  }
  m[kQZero] = (double)nz;
  m[kQBad] = (double)nbad;
  block_sum<kNormQ, kPassWaves>(m, sh);
  double *out = partials + out_buf * kPartStride * kMaxPartialBlocks;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kNormQ; ++k) out[blockIdx.x * kPartStride + k] = m[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // from LDS: the state is not held in registers across the pass
    NormState o = shs;
    o.pending = 0;
    o.buf = out_buf;
    o.nparts = gridDim.x;
    *st_out = o;
  }
}

// Last step (from the last pass's moments unless already converged), then
// tau' = A tau and F = exp(-tau').
__global__ __launch_bounds__(kNormThreads) void norm_finalise_kernel(
    float *__restrict__ tau, float *__restrict__ F, int64_t P, const double *partials,
    const NormState *st_prev, NormState *st_out, double *A_dev, uint32_t *status) {
  __shared__ double sh[block_sum_lds(kNormQ, kNormWaves)];
  __shared__ NormState shs;
  if (threadIdx.x == 0) shs = *st_prev;
  __syncthreads();
  if (!shs.done) {
    if (shs.pending) {  // no moments at A: the cap on passes was hit
      if (threadIdx.x == 0) {
        shs.done = 1;
        shs.status |= LYAF_STATUS_NOCONV;
      }
    } else {  // one more step from the last pass's moments
      double tot[kNormQ];
      reduce_partials<kNormQ, kNormWaves>(partials + shs.buf * kPartStride * kMaxPartialBlocks,
                                          shs.nparts, tot, sh);
      if (threadIdx.x == 0) {
        NormState s = norm_step(shs, tot);
        // accepted: converged in the exact phase, or a domain / no-root
        // verdict, or an FP32-phase step as small as the exact acceptance
        const bool accepted = s.done || s.step <= kNormAcceptStep;
        s.done = 1;
        if (!accepted) s.status |= LYAF_STATUS_NOCONV;
        shs = s;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *st_out = shs;
    *A_dev = shs.A;
    if (shs.status) atomicOr(status, (uint32_t)shs.status);
  }
  const double A = shs.A;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((reinterpret_cast<uintptr_t>(tau) & 15) == 0 &&
      (F == nullptr || (reinterpret_cast<uintptr_t>(F) & 15) == 0)) {
    const int64_t P4 = P >> 2;
    float4 *t4 = reinterpret_cast<float4 *>(tau);
    float4 *f4 = reinterpret_cast<float4 *>(F);
    for (int64_t p = base; p < P4; p += stride) {
      const float4 t = t4[p];
      float4 o;
      o.x = (float)(A * (double)t.x);
      o.y = (float)(A * (double)t.y);
      o.z = (float)(A * (double)t.z);
      o.w = (float)(A * (double)t.w);
      t4[p] = o;
      if (F) f4[p] = make_float4(expf(-o.x), expf(-o.y), expf(-o.z), expf(-o.w));
    }
    for (int64_t p = (P4 << 2) + base; p < P; p += stride) {
      const float ts = (float)(A * (double)tau[p]);
      tau[p] = ts;
      if (F) F[p] = expf(-ts);
    }
  } else {
    for (int64_t p = base; p < P; p += stride) {
      const float ts = (float)(A * (double)tau[p]);
      tau[p] = ts;
      if (F) F[p] = expf(-ts);
    }
  }
}

static int norm_grid(int64_t pixels) {  // backward reductions
  int64_t g = (pixels + kNormThreads * 16 - 1) / (kNormThreads * 16);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxPartialBlocks));
}

hipError_t launch_norm_buffers(int64_t n_pix, float *tau, float *F, double target_F,
                               double *A_dev, double *partials, NormState *norm,
                               uint32_t *status, hipStream_t st) {
  int64_t g = (n_pix + kPassThreads * 16 - 1) / (kPassThreads * 16);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxPartialBlocks));
  float *sample = reinterpret_cast<float *>(partials + 2 * kPartStride * kMaxPartialBlocks);
  hipLaunchKernelGGL(norm_gather_kernel, dim3(kSampleN / kGatherThreads), dim3(kGatherThreads),
                     0, st, tau, n_pix, sample);
  hipLaunchKernelGGL(norm_sample_kernel, dim3(1), dim3(kSampleThreads), 0, st, sample, n_pix,
                     target_F, norm);
  for (int k = 0; k < kNormPasses; ++k)
    hipLaunchKernelGGL(norm_pass_kernel, dim3(grid), dim3(kPassThreads), 0, st, tau, n_pix,
                       partials, norm + k, norm + k + 1, status);
  const int fgrid = (int)std::min<int64_t>((n_pix + 4095) / 4096, 2048);
  hipLaunchKernelGGL(norm_finalise_kernel, dim3(std::max(fgrid, 1)), dim3(kNormThreads), 0, st,
                     tau, F, n_pix, partials, norm + kNormPasses, norm + kNormPasses + 1, A_dev,
                     status);
  return hipGetLastError();
}

hipError_t launch_norm(int64_t n_pix, float *tau, float *F, double target_F, double *A_dev,
                       Workspace &ws, hipStream_t st) {
  return launch_norm_buffers(n_pix, tau, F, target_F, A_dev, ws.partials, ws.norm, ws.status,
                             st);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the root-find's scratch (the FP64 partials of two
// passes and room for the sample, the iteration states, and a status word for
// callers that pass none) lives in one file-scope device array instead of
// a workspace.  The passes use at most kMaxPartialBlocks workgroups and a
// fixed sample whatever n_pix is, so this fixed size serves every batch.  In
// host code `scratch` names a host-side stand-in, not device memory: the
// device address comes from hipGetSymbolAddress, once per device (each device
// holds its own copy of the array).
constexpr size_t kNoAllocPartialsBytes = sizeof(double) * (size_t)kPartialsDoubles;
constexpr size_t kNoAllocStatesOffset = (kNoAllocPartialsBytes + 255) / 256 * 256;
constexpr size_t kNoAllocStatusOffset =
    (kNoAllocStatesOffset + sizeof(NormState) * (kNormPasses + 2) + 255) / 256 * 256;
constexpr size_t kNoAllocScratchBytes = kNoAllocStatusOffset + 256;
static_assert(kNoAllocScratchBytes == kNormNoAllocScratchBytes,
              "scratch size declared in lyaf_internal.h");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

hipError_t norm_noalloc_scratch(void **ptr_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr_out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_norm_noalloc(int64_t n_pix, float *tau, float *F, double target_F,
                               double *A_dev, uint32_t *status, hipStream_t st) {
  void *base = nullptr;
  hipError_t e = norm_noalloc_scratch(&base);
  if (e != hipSuccess) return e;
  unsigned char *b = static_cast<unsigned char *>(base);
  double *partials = reinterpret_cast<double *>(b);
  NormState *norm = reinterpret_cast<NormState *>(b + kNoAllocStatesOffset);
  uint32_t *st_word = status ? status : reinterpret_cast<uint32_t *>(b + kNoAllocStatusOffset);
  return launch_norm_buffers(n_pix, tau, F, target_F, A_dev, partials, norm, st_word, st);
}

// ---------------------------------------------------------------------------
// Backward.  G_p = gT_p - F_p gF_p with F_p = exp(-A tau_p) as in the forward;
// implicit A adds -A F_p (sum G tau)/(sum F tau).
__device__ __forceinline__ void fwd_F(double A, float t, float &ts, float &Fp) {
  ts = (float)(A * (double)t);
  Fp = expf(-ts);
}

__global__ __launch_bounds__(kNormThreads) void normbw_reduce_kernel(
    const float *__restrict__ tau, const double *A_dev, const float *__restrict__ gF,
    const float *__restrict__ gT, int64_t P, double *partials) {
  __shared__ double sh[block_sum_lds(2, kNormWaves)];
  const double A = *A_dev;
  double v[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    float ts, Fp;
    fwd_F(A, tau[p], ts, Fp);
    const float G = (gT ? gT[p] : 0.f) - Fp * (gF ? gF[p] : 0.f);
    v[0] += (double)G * (double)tau[p];
    v[1] += (double)Fp * (double)tau[p];
  }
  block_sum<2, kNormWaves>(v, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * kPartStride + 0] = v[0];
    partials[blockIdx.x * kPartStride + 1] = v[1];
  }
}

__global__ __launch_bounds__(kNormThreads) void normbw_ratio_kernel(int nblocks,
                                                                    const double *partials,
                                                                    double *ratio) {
  __shared__ double sh[block_sum_lds(2, kNormWaves)];
  double tot[2];
  reduce_partials<2, kNormWaves>(partials, nblocks, tot, sh);
  if (threadIdx.x == 0) *ratio = (tot[1] != 0.0) ? tot[0] / tot[1] : 0.0;
}

__global__ __launch_bounds__(kNormThreads) void normbw_apply_kernel(
    const float *__restrict__ tau, const double *A_dev, const float *__restrict__ gF,
    const float *__restrict__ gT, int64_t P, const double *ratio, int implicit_A,
    float *__restrict__ out) {
  const double A = *A_dev;
  const float Af = (float)A;
  const float rA = implicit_A ? (float)(A * *ratio) : 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    float ts, Fp;
    fwd_F(A, tau[p], ts, Fp);
    const float G = (gT ? gT[p] : 0.f) - Fp * (gF ? gF[p] : 0.f);
    out[p] = Af * G - rA * Fp;
  }
}

hipError_t launch_norm_backward(int64_t n_pix, const float *tau, const double *A_dev,
                                const float *gF, const float *gT, int implicit_A, float *out,
                                Workspace &ws, hipStream_t st) {
  const int grid = norm_grid(n_pix);
  if (implicit_A) {
    hipLaunchKernelGGL(normbw_reduce_kernel, dim3(grid), dim3(kNormThreads), 0, st, tau, A_dev,
                       gF, gT, n_pix, ws.partials);
    hipLaunchKernelGGL(normbw_ratio_kernel, dim3(1), dim3(kNormThreads), 0, st, grid,
                       ws.partials, ws.ratio);
  }
  const int fgrid = (int)std::min<int64_t>((n_pix + 1023) / 1024 + 1, 65536);
  hipLaunchKernelGGL(normbw_apply_kernel, dim3(fgrid), dim3(kNormThreads), 0, st, tau, A_dev,
                     gF, gT, n_pix, ws.ratio, implicit_A, out);
  return hipGetLastError();
}

}  // namespace lyaf
