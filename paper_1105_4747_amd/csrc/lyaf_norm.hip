// lyaf_norm.hip -- mean-flux renormalisation of Section 2.3 (Greig, Bolton &
// Wyithe 2011): find A with (1/P) sum_p exp(-A tau_p) = target_F over all
// pixels, then tau' = A tau and F = exp(-tau'); plus its backward pass.
//
// The root-find runs on the device without host synchronisation: one pass
// (norm_init) forms sum tau, the count of tau = 0 pixels and the domain check,
// and starts from the Jensen lower bound A0 = -ln F / <tau> (g(A0) >= 0, and g
// is convex and decreasing, so Newton steps from the left never overshoot).
// Each further pass (norm_moments) evaluates S_k = sum tau^k exp(-A tau),
// k = 0, 1, 2, in FP64 per workgroup; a one-workgroup kernel (norm_update)
// sums the partials and applies a safeguarded Halley step (Newton, then
// bisection, as fallbacks) inside the bracket.  A kernel boundary, not a
// device-scope fence, publishes the partials: on a multi-XCD part a fence per
// workgroup writes back and invalidates L2 and serialises the pass.  A fixed
// number of passes is enqueued; once converged the remaining ones return at
// once.  Partial sums are combined in a fixed order, so results are bitwise
// reproducible.
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    const float t = tau[p];
    if (!(t >= 0.f) || !isfinite(t)) v[2] += 1.0;
    else {
      v[0] += (double)t;
      v[1] += (t == 0.f) ? 1.0 : 0.0;
    }
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = v[0];
    partials[blockIdx.x * 4 + 1] = v[1];
    partials[blockIdx.x * 4 + 2] = v[2];
  }
}

// One workgroup: fixed-order sum of the init partials, starting state.
__global__ __launch_bounds__(kNormThreads) void norm_start_kernel(int nblocks, int64_t P,
                                                                  double target, NormState *st,
                                                                  const double *partials,
                                                                  uint32_t *status) {
  __shared__ double sh[16];
  double tot[3];
  reduce_partials<3>(partials, nblocks, tot, sh);
  if (threadIdx.x == 0) {
    const double Pd = (double)P;
    NormState s;
    s.P = Pd;
    s.target = target;
    s.iter = 0;
    s.done = 0;
    s.status = 0;
    s.pad = 0;
    s.lo = 0.0;
    s.hi = INFINITY;
    s.A = -log(target) / (tot[0] / Pd);  // Jensen: g(A0) >= 0
    if (tot[2] > 0.0) {
      s.done = 1;
      s.status = LYAF_STATUS_DOMAIN;
    } else if (!(tot[1] / Pd < target)) {
      s.done = 1;
      s.status = LYAF_STATUS_NOROOT;
    }
    *st = s;
    if (s.status) atomicOr(status, (uint32_t)s.status);
  }
}

// One pass: S_k = sum tau^k exp(-A tau), k = 0..2, per workgroup.
__global__ __launch_bounds__(kNormThreads) void norm_moments_kernel(const float *__restrict__ tau,
                                                                    int64_t P, const NormState *st,
                                                                    double *partials) {
  __shared__ double sh[16];
  if (st->done) return;  // converged (or failed) in an earlier pass
  const double A = st->A;
  double v[3] = {0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((reinterpret_cast<uintptr_t>(tau) & 15) == 0) {
    const int64_t P4 = P >> 2;
    const float4 *t4 = reinterpret_cast<const float4 *>(tau);
    for (int64_t p = base; p < P4; p += stride) {
      const float4 q = t4[p];
      const double t[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double e = exp_neg(A * t[k]);
        const double te = t[k] * e;
        v[0] += e;
        v[1] += te;
        v[2] = fma(te, t[k], v[2]);
      }
    }
    for (int64_t p = (P4 << 2) + base; p < P; p += stride) {
      const double t = tau[p];
      const double e = exp_neg(A * t);
      v[0] += e;
      v[1] += t * e;
      v[2] = fma(t * e, t, v[2]);
    }
  } else {
    for (int64_t p = base; p < P; p += stride) {
      const double t = tau[p];
      const double e = exp_neg(A * t);
      v[0] += e;
      v[1] += t * e;
      v[2] = fma(t * e, t, v[2]);
    }
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = v[0];
    partials[blockIdx.x * 4 + 1] = v[1];
    partials[blockIdx.x * 4 + 2] = v[2];
  }
}

// One workgroup: fixed-order sum of the moment partials and one safeguarded
// Halley step inside the bracket.
__global__ __launch_bounds__(kNormThreads) void norm_update_kernel(int nblocks, NormState *st,
                                                                   const double *partials,
                                                                   uint32_t *status) {
  __shared__ double sh[16];
  if (st->done) return;
  double tot[3];
  reduce_partials<3>(partials, nblocks, tot, sh);
  if (threadIdx.x == 0) {
    NormState s = *st;
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
      conv = fabs(An - s.A) <= 1e-12 * An;
    }
    s.A = An;
    s.iter += 1;
    if (conv) {
      s.done = 1;
    } else if (s.iter >= kNormMaxIter) {
      s.done = 1;
      s.status = LYAF_STATUS_NOCONV;
      atomicOr(status, (uint32_t)LYAF_STATUS_NOCONV);
    }
    *st = s;
  }
}

__global__ __launch_bounds__(kNormThreads) void norm_finalise_kernel(float *__restrict__ tau,
                                                                     float *__restrict__ F,
                                                                     int64_t P,
                                                                     const NormState *st,
                                                                     double *A_dev) {
  const double A = st->A;
  if (blockIdx.x == 0 && threadIdx.x == 0) *A_dev = A;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    const float ts = (float)(A * (double)tau[p]);
    tau[p] = ts;
    if (F) F[p] = expf(-ts);
  }
}

static int norm_grid(int64_t P) {
  int64_t g = (P + kNormThreads * 8 - 1) / (kNormThreads * 8);
  if (g < 1) g = 1;
  if (g > kMaxPartialBlocks) g = kMaxPartialBlocks;
  return (int)g;
}

hipError_t launch_norm(int64_t n_pix, float *tau, float *F, double target_F, double *A_dev,
                       Workspace &ws, hipStream_t st) {
  const int grid = norm_grid(n_pix);
  hipLaunchKernelGGL(norm_init_kernel, dim3(grid), dim3(kNormThreads), 0, st, tau, n_pix,
                     ws.partials);
  hipLaunchKernelGGL(norm_start_kernel, dim3(1), dim3(kNormThreads), 0, st, grid, n_pix,
                     target_F, ws.norm, ws.partials, ws.status);
  for (int it = 0; it < kNormMaxIter; ++it) {
    hipLaunchKernelGGL(norm_moments_kernel, dim3(grid), dim3(kNormThreads), 0, st, tau, n_pix,
                       ws.norm, ws.partials);
    hipLaunchKernelGGL(norm_update_kernel, dim3(1), dim3(kNormThreads), 0, st, grid, ws.norm,
                       ws.partials, ws.status);
  }
  const int fgrid = (int)std::min<int64_t>((n_pix + 1023) / 1024 + 1, 65536);
  hipLaunchKernelGGL(norm_finalise_kernel, dim3(fgrid), dim3(kNormThreads), 0, st, tau, F,
                     n_pix, ws.norm, A_dev);
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
