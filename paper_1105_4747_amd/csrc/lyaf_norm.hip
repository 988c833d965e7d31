// lyaf_norm.hip -- mean-flux renormalisation of Section 2.3 (Greig, Bolton &
// Wyithe 2011): find A with (1/P) sum_p exp(-A tau_p) = target_F over all
// pixels, then tau' = A tau and F = exp(-tau'); plus its backward pass.
//
// The root-find runs on the device without host synchronisation: one pass
// (norm_init) forms sum tau, the count of tau = 0 pixels and the domain check,
// and starts from the Jensen lower bound A0 = -ln F / <tau> (g(A0) >= 0, and g
// is convex and decreasing, so Newton steps from the left never overshoot).
// Each further pass evaluates S_k = sum tau^k exp(-A tau), k = 0, 1, 2, in FP64
// per workgroup.  The next pass (or the finalise kernel) begins with every
// workgroup summing those partials in the same fixed order and taking the
// same safeguarded Halley step (Newton, then bisection, as fallbacks) inside
// the bracket.  A kernel boundary, not a device-scope fence, publishes the
// partials: on a multi-XCD part a fence per workgroup writes back and
// invalidates L2 and serialises the pass.  A fixed number of passes is
// enqueued; once converged the remaining ones return at once.  Results are
// bitwise reproducible.
#include <math.h>

#include "lyaf_internal.h"

namespace lyaf {

// exp(-x) for x >= 0 in FP64: Cody-Waite reduction x = k ln2 + r with
// |r| <= ln2/2 (ln2 split into a 32-bit head and a tail so k*ln2_hi is exact),
// then the Taylor series of exp(-r) to degree 13 (truncation below 1e-17).
__device__ __forceinline__ double exp_neg(double x) {
  if (!(x <= 745.2)) return 0.0;
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double k = rint(x * kLog2e);
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
  return ldexp(p, -(int)k);
}

// exp(-x) for x >= 0 with FP64 argument reduction and the FP32 hardware
// exp2 on the fraction: x log2 e = n + f, f in [0, 1), result 2^-n * 2^-f.
// Relative error below 1e-7 (rounding f to FP32 and the exp2 unit); used for
// the approach iterations only.
__device__ __forceinline__ double exp_neg_fast(double y /* = x log2 e */) {
  if (!(y <= 1074.0)) return 0.0;
  const double nf = floor(y);
  const float f = (float)(y - nf);
  return ldexp((double)__builtin_amdgcn_exp2f(-f), -(int)nf);
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *sh /*[N*4]*/) {
#pragma unroll
  for (int q = 0; q < N; ++q)
    for (int m = 32; m >= 1; m >>= 1) v[q] += __shfl_xor(v[q], m);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) sh[q * 4 + w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = (sh[q * 4 + 0] + sh[q * 4 + 1]) + (sh[q * 4 + 2] + sh[q * 4 + 3]);
  __syncthreads();
}

// Fixed-order reduction of NQ partial quantities written per workgroup.
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double *partials, int nblocks,
                                                double (&tot)[NQ], double *sh) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) tot[q] = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += blockDim.x)
#pragma unroll
    for (int q = 0; q < NQ; ++q) tot[q] += partials[k * 4 + q];
  block_sum<NQ>(tot, sh);
}

constexpr int kNormThreads = 256;

// Pass 0: sum tau, count tau == 0 and count invalid values, per workgroup.
__global__ __launch_bounds__(kNormThreads) void norm_init_kernel(const float *__restrict__ tau,
                                                                 int64_t P, double *partials) {
  __shared__ double sh[16];
  double v[3] = {0.0, 0.0, 0.0};  // sum tau, #zeros, #bad
  auto add = [&](float t) {
    if (!(t >= 0.f) || !isfinite(t)) v[2] += 1.0;
    else {
      v[0] += (double)t;
      v[1] += (t == 0.f) ? 1.0 : 0.0;
    }
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done_to = 0;
  if ((reinterpret_cast<uintptr_t>(tau) & 15) == 0) {
    const int64_t P4 = P >> 2;
    const float4 *t4 = reinterpret_cast<const float4 *>(tau);
    int64_t p = base;
    for (; p + stride < P4; p += 2 * stride) {
      const float4 qa = t4[p], qb = t4[p + stride];
      add(qa.x); add(qa.y); add(qa.z); add(qa.w);
      add(qb.x); add(qb.y); add(qb.z); add(qb.w);
    }
    for (; p < P4; p += stride) {
      const float4 qa = t4[p];
      add(qa.x); add(qa.y); add(qa.z); add(qa.w);
    }
    done_to = P4 << 2;
  }
  for (int64_t p = done_to + base; p < P; p += stride) add(tau[p]);
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = v[0];
    partials[blockIdx.x * 4 + 1] = v[1];
    partials[blockIdx.x * 4 + 2] = v[2];
  }
}

// Starting state from the pass-0 sums: the Jensen lower bound
// A0 = -ln F / <tau> (g(A0) >= 0), or a terminal state with a status bit.
__device__ NormState norm_start(const double (&tot)[3], double P, double target) {
  NormState s;
  s.P = P;
  s.target = target;
  s.iter = 0;
  s.done = 0;
  s.status = 0;
  s.exact = 0;
  s.lo = 0.0;
  s.hi = INFINITY;
  s.A = -log(target) / (tot[0] / P);
  if (tot[2] > 0.0) {
    s.done = 1;
    s.status = LYAF_STATUS_DOMAIN;
  } else if (!(tot[1] / P < target)) {
    s.done = 1;
    s.status = LYAF_STATUS_NOROOT;
  }
  return s;
}

// One safeguarded Halley step from the moments S0, S1, S2 at s.A.
__device__ NormState norm_step(NormState s, const double (&tot)[3]) {
  const double g = tot[0] / s.P - s.target;  // g(A) = <exp(-A tau)> - F
  const double g1 = -tot[1] / s.P;           // g'(A)
  const double g2 = tot[2] / s.P;            // g''(A)
  double An = s.A;
  bool conv = false;
  if (g == 0.0) {
    conv = true;
  } else {
    if (g > 0.0) s.lo = s.A; else s.hi = s.A;
    const double den = 2.0 * g1 * g1 - g * g2;
    const double halley = (den != 0.0) ? s.A - 2.0 * g * g1 / den : NAN;
    const double newton = (g1 < 0.0) ? s.A - g / g1 : NAN;
    if (halley > s.lo && halley < s.hi) An = halley;
    else if (newton > s.lo && newton < s.hi) An = newton;
    else if (isfinite(s.hi)) An = 0.5 * (s.lo + s.hi);
    else An = 2.0 * s.A;
    // Halley converges cubically: once a step is below kNormAcceptStep of A
    // the iterate it produces is within ~K 1e-15 of the root (K, the ratio of
    // successive errors to the cube, is below 0.1 on lognormal-field tau),
    // so it is accepted without another pass.
    conv = fabs(An - s.A) <= kNormAcceptStep * An;
  }
  s.A = An;
  s.iter += 1;
  if (conv) {
    // the approach used FP32 exponentials: finish with exact FP64 moments.
    // Signs of g seen in the approach can be wrong within its ~1e-7 error,
    // so the exact phase starts from an open bracket.
    if (s.exact) {
      s.done = 1;
    } else {
      s.exact = 1;
      s.lo = 0.0;
      s.hi = INFINITY;
    }
  }
  return s;
}

// Pass k >= 1.  Every workgroup sums the previous pass's partials in the same
// fixed order and takes the same step, so no update kernel and no
// device-scope fence are needed; workgroup 0 records the state.  Then, unless
// the iteration has finished, S_k = sum tau^k exp(-A tau), k = 0..2, at the
// new A, per workgroup.
__global__ __launch_bounds__(kNormThreads) void norm_pass_kernel(
    int pass, const float *__restrict__ tau, int64_t P, double target,
    const double *__restrict__ part_in, double *__restrict__ part_out,
    const NormState *st_prev, NormState *st_out, uint32_t *status) {
  __shared__ double sh[16];
  __shared__ NormState shs;
  if (threadIdx.x == 0) shs = (pass == 1) ? NormState{} : *st_prev;
  __syncthreads();
  if (pass > 1 && shs.done) {  // finished in an earlier pass
    if (blockIdx.x == 0 && threadIdx.x == 0) *st_out = shs;
    return;
  }
  double tot[3];
  reduce_partials<3>(part_in, gridDim.x, tot, sh);
  if (threadIdx.x == 0) {
    const NormState s = (pass == 1) ? norm_start(tot, (double)P, target) : norm_step(shs, tot);
    shs = s;
    if (blockIdx.x == 0) {
      *st_out = s;
      if (pass == 1 && s.status) atomicOr(status, (uint32_t)s.status);
    }
  }
  __syncthreads();
  if (shs.done) return;
  const double A = shs.A;
  const double Al = shs.A * kLog2e;
  const bool exact = shs.exact != 0;
  double v[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
  // two accumulator sets (elements alternate) halve the FP64 add chain
  auto add2 = [&](double t, double (&a)[3]) {
    const double e = exact ? exp_neg(A * t) : exp_neg_fast(Al * t);
    const double te = t * e;
    a[0] += e;
    a[1] += te;
    a[2] = fma(te, t, a[2]);
  };
  auto add = [&](double t) { add2(t, v); };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done_to = 0;
  if ((reinterpret_cast<uintptr_t>(tau) & 15) == 0) {
    const int64_t P4 = P >> 2;
    const float4 *t4 = reinterpret_cast<const float4 *>(tau);
    int64_t p = base;
    for (; p + stride < P4; p += 2 * stride) {  // two loads in flight
      const float4 qa = t4[p], qb = t4[p + stride];
      add2(qa.x, v); add2(qa.y, u); add2(qa.z, v); add2(qa.w, u);
      add2(qb.x, v); add2(qb.y, u); add2(qb.z, v); add2(qb.w, u);
    }
    for (; p < P4; p += stride) {
      const float4 qa = t4[p];
      add2(qa.x, v); add2(qa.y, u); add2(qa.z, v); add2(qa.w, u);
    }
    done_to = P4 << 2;
  }
  for (int64_t p = done_to + base; p < P; p += stride) add((double)tau[p]);
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] += u[k];
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    part_out[blockIdx.x * 4 + 0] = v[0];
    part_out[blockIdx.x * 4 + 1] = v[1];
    part_out[blockIdx.x * 4 + 2] = v[2];
  }
}

// Last step (from the last pass's moments unless already converged), then
// tau' = A tau and F = exp(-tau').
__global__ __launch_bounds__(kNormThreads) void norm_finalise_kernel(
    float *__restrict__ tau, float *__restrict__ F, int64_t P, int nparts,
    const double *__restrict__ part_in, const NormState *st_prev, NormState *st_out,
    double *A_dev, uint32_t *status) {
  __shared__ double sh[16];
  __shared__ NormState shs;
  if (threadIdx.x == 0) shs = *st_prev;
  __syncthreads();
  if (!shs.done) {  // one more step from the last pass's moments
    double tot[3];
    reduce_partials<3>(part_in, nparts, tot, sh);
    if (threadIdx.x == 0) {
      NormState s = norm_step(shs, tot);
      // accepted if the step was small (then norm_step either finished or
      // moved to the exact phase); otherwise the cap on passes was hit
      const bool accepted = s.done || s.exact != shs.exact;
      s.done = 1;
      if (!accepted) s.status |= LYAF_STATUS_NOCONV;
      shs = s;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *st_out = shs;
    *A_dev = shs.A;
    if (shs.status & LYAF_STATUS_NOCONV) atomicOr(status, (uint32_t)LYAF_STATUS_NOCONV);
  }
  const double A = shs.A;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    const float ts = (float)(A * (double)tau[p]);
    tau[p] = ts;
    if (F) F[p] = expf(-ts);
  }
}

static int norm_grid(int64_t P) {
  int64_t g = (P + kNormThreads * 16 - 1) / (kNormThreads * 16);
  if (g < 1) g = 1;
  if (g > kMaxPartialBlocks) g = kMaxPartialBlocks;
  return (int)g;
}

hipError_t launch_norm(int64_t n_pix, float *tau, float *F, double target_F, double *A_dev,
                       Workspace &ws, hipStream_t st) {
  const int grid = norm_grid(n_pix);
  double *part[2] = {ws.partials, ws.partials + 4 * kMaxPartialBlocks};
  hipLaunchKernelGGL(norm_init_kernel, dim3(grid), dim3(kNormThreads), 0, st, tau, n_pix,
                     part[0]);
  for (int k = 1; k <= kNormMaxIter; ++k)
    hipLaunchKernelGGL(norm_pass_kernel, dim3(grid), dim3(kNormThreads), 0, st, k, tau, n_pix,
                       target_F, part[(k - 1) & 1], part[k & 1], ws.norm + (k - 1),
                       ws.norm + k, ws.status);
  const int fgrid = (int)std::min<int64_t>((n_pix + 2047) / 2048, 2048);
  hipLaunchKernelGGL(norm_finalise_kernel, dim3(std::max(fgrid, 1)), dim3(kNormThreads), 0, st,
                     tau, F, n_pix, grid, part[kNormMaxIter & 1], ws.norm + kNormMaxIter,
                     ws.norm + kNormMaxIter + 1, A_dev, ws.status);
  return hipGetLastError();
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
  __shared__ double sh[16];
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
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = v[0];
    partials[blockIdx.x * 4 + 1] = v[1];
  }
}

__global__ __launch_bounds__(kNormThreads) void normbw_ratio_kernel(int nblocks,
                                                                    const double *partials,
                                                                    double *ratio) {
  __shared__ double sh[16];
  double tot[2];
  reduce_partials<2>(partials, nblocks, tot, sh);
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
