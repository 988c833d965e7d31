// lyaf_fft.h -- in-LDS complex FFT passes shared by the kernels that transform
// along one axis (the 1D flux power spectrum, the skewer-only field synthesis,
// the 3D flux power spectrum).  Device code only; nothing here is public ABI.
//
// A batch of C transforms of N points (N, C powers of two) sits in LDS with
// element j of transform c at buf[j C + c], so that C consecutive columns of a
// global array load and store without bank conflicts.  Each Stockham pass of
// radix R reads, for butterfly (j, c) with k = j mod Ns, the R inputs
// x_r = buf[(j + r N/R) C + c], twiddles x_r by w^r, w = e^{-2 pi i k/(R Ns)},
// and after a barrier writes their length-R DFT to buf[((j - k) R + k + r Ns) C + c];
// passes of radix 8 run while 8 Ns <= N, then one of radix 4 or 2 as log2 N
// needs.  Every thread holds its butterflies' outputs in registers across the
// barrier, so the passes work in place.  The transforms are forward
// (e^{-2 pi i}); an inverse transform is the conjugate of the forward
// transform of the conjugate, which the callers apply on the way in and out.
//
// Twiddles come from one half-period table of the largest transform,
// T[t] = e^{-2 pi i t / kFftTableLen} for t < kFftTableLen / 2, held in FP64 in
// device memory (it stays in L1/L2); a transform of N points takes every
// (kFftTableLen / N)-th entry.  FP32 batches round the entry once.
#pragma once

#include <hip/hip_runtime.h>

namespace lyaf {

constexpr int kFftTableLen = 4096;  // longest transform the table serves

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i and by +i
__device__ inline double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }
__device__ inline float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ inline double2 mul_pi(double2 a) { return make_double2(-a.y, a.x); }
__device__ inline float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }
__device__ inline double2 conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline float2 conj(float2 a) { return make_float2(a.x, -a.y); }

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations (lgkmcnt(0); vmcnt and expcnt left at their maxima, encoding
// 0xC07F on gfx9-family parts), then s_barrier.  Unlike __syncthreads() it
// does not wait for global loads, so reads of the next tile issued before it
// stay in flight across the transform's passes.  The empty asm statements keep
// the compiler from moving memory accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <typename V>
__device__ inline V twiddle_as(double2 w);
template <>
__device__ inline double2 twiddle_as<double2>(double2 w) { return w; }
template <>
__device__ inline float2 twiddle_as<float2>(double2 w) {
  return make_float2((float)w.x, (float)w.y);
}

template <typename V>
__device__ inline void dft4(V a0, V a1, V a2, V a3, V &y0, V &y1, V &y2, V &y3) {
  const V s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const V s13 = cadd(a1, a3), d13 = csub(a1, a3);
  y0 = cadd(s02, s13);
  y1 = cadd(d02, mul_mi(d13));
  y2 = csub(s02, s13);
  y3 = cadd(d02, mul_pi(d13));
}

// One in-place pass of radix R over C = 2^lgC transforms of N points (see the
// header).  CAP bounds N C over every call of the instantiation, so each of
// the THREADS threads holds at most CAP / (R THREADS) butterflies.  A length-8
// DFT is two length-4 DFTs of x_k + x_{k+4} and (x_k - x_{k+4}) e^{-2 pi i k/8}.
template <int R, int THREADS, int CAP, typename V>
__device__ void fft_pass(V *buf, const double2 *__restrict__ T, int N, int lgC, int Ns) {
  using S = decltype(V{}.x);
  constexpr int B = (CAP / R + THREADS - 1) / THREADS;
  const int nb = (N / R) << lgC;
  const int cmask = (1 << lgC) - 1;
  const int step = kFftTableLen / (R * Ns);  // stride in the table
  V y[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int q = (int)threadIdx.x + b * THREADS;
    if (q < nb) {
      const int c = q & cmask;
      const int j = q >> lgC;
      const int k = j & (Ns - 1);
      const V w = twiddle_as<V>(T[k * step]);
      V x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = buf[((j + r * (N / R)) << lgC) + c];
      if constexpr (R == 8) {
        const V w2 = cmul(w, w), w3 = cmul(w2, w), w4 = cmul(w2, w2);
        const V w5 = cmul(w4, w), w6 = cmul(w3, w3), w7 = cmul(w6, w);
        x[1] = cmul(x[1], w);
        x[2] = cmul(x[2], w2);
        x[3] = cmul(x[3], w3);
        x[4] = cmul(x[4], w4);
        x[5] = cmul(x[5], w5);
        x[6] = cmul(x[6], w6);
        x[7] = cmul(x[7], w7);
        constexpr S h = (S)0.70710678118654752440;  // sqrt(1/2)
        const V b0 = csub(x[0], x[4]);
        const V t1 = csub(x[1], x[5]);
        V b1;  // * (1 - i)/sqrt2
        b1.x = h * (t1.x + t1.y);
        b1.y = h * (t1.y - t1.x);
        const V b2 = mul_mi(csub(x[2], x[6]));
        const V t3 = csub(x[3], x[7]);
        V b3;  // * -(1 + i)/sqrt2
        b3.x = h * (t3.y - t3.x);
        b3.y = -h * (t3.x + t3.y);
        dft4(cadd(x[0], x[4]), cadd(x[1], x[5]), cadd(x[2], x[6]), cadd(x[3], x[7]), y[b][0],
             y[b][2], y[b][4], y[b][6]);
        dft4(b0, b1, b2, b3, y[b][1], y[b][3], y[b][5], y[b][7]);
      } else if constexpr (R == 4) {
        const V w2 = cmul(w, w), w3 = cmul(w2, w);
        dft4(x[0], cmul(x[1], w), cmul(x[2], w2), cmul(x[3], w3), y[b][0], y[b][1], y[b][2],
             y[b][3]);
      } else {
        const V a1 = cmul(x[1], w);
        y[b][0] = cadd(x[0], a1);
        y[b][1] = csub(x[0], a1);
      }
    }
    // one butterfly's inputs live at a time: without this the compiler reads
    // every butterfly's inputs first and runs out of registers at large B
    asm volatile("" ::: "memory");
  }
  lds_barrier();  // every read of this pass is done
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int q = (int)threadIdx.x + b * THREADS;
    if (q < nb) {
      const int c = q & cmask;
      const int j = q >> lgC;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[((base + r * Ns) << lgC) + c] = y[b][r];
    }
  }
  lds_barrier();
}

// The whole forward transform of the batch (N >= 1; N = 1 is the identity).
// The caller has published buf with a barrier; the last pass ends with one
// (LDS only: global loads issued before the transform may still be in flight).
template <int THREADS, int CAP, typename V>
__device__ void fft_batch(V *buf, const double2 *__restrict__ T, int N, int lgC) {
  int Ns = 1;
  while (Ns * 8 <= N) {
    fft_pass<8, THREADS, CAP>(buf, T, N, lgC, Ns);
    Ns *= 8;
  }
  if (Ns * 4 <= N) {
    fft_pass<4, THREADS, CAP>(buf, T, N, lgC, Ns);
    Ns *= 4;
  }
  if (Ns * 2 <= N) fft_pass<2, THREADS, CAP>(buf, T, N, lgC, Ns);
}

}  // namespace lyaf
