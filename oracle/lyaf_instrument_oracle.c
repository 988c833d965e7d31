/*
 * lyaf_instrument_oracle.c -- plain FP64 CPU oracle for the instrument model
 * applied to the transmitted flux.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no header, constant or helper with the HIP
 * library (nor with lyaf_oracle.c): every constant and formula is written out
 * here from the paper (Greig, Bolton & Wyithe 2011).
 *
 * The paper turns each simulated flux spectrum into a mock observation in
 * three steps (Section 3.1 for the high-resolution spectra: FWHM 7 km/s,
 * 0.05 A bins, S/N ~ 50; Section 3.2 for the BOSS-like spectra: FWHM ~3.63 A
 * ~ 224 km/s, 1.0375 A bins, S/N = 5, restricted to the quasar's Lya-Lyb
 * path minus 3000 km/s; Section 4 for the SDSS-like flux PDF: FWHM 170 km/s,
 * ~1 A bins, S/N = 3.8):
 *
 *   1. Convolution with a Gaussian line-spread function of full width at half
 *      maximum FWHM.  On the periodic grid of N pixels of width dv this is
 *        Fc_i = sum_{j=0}^{N-1} c_{(i-j) mod N} F_j,
 *        c_o = g(d_o) / sum_{o'} g(d_o'),  g(d) = exp(-(d / b_L)^2),
 *        b_L = FWHM / (2 sqrt(ln 2)),
 *      with d_o the minimal image of o*dv in [-V/2, V/2), V = N dv.  The
 *      weights sum to one, so a flat spectrum stays flat.  FWHM = 0 means no
 *      convolution (c_0 = 1).
 *
 *   2. Resampling onto bins of width dv_bin.  Pixel i covers velocities
 *      [(i - 1/2) dv, (i + 1/2) dv) and carries the constant value Fc_i; bin k
 *      of a skewer covers [v_start + k dv_bin, v_start + (k+1) dv_bin) (taken
 *      periodically) and its value is the average of that piecewise-constant
 *      spectrum over the bin.  In pixel coordinates x = v/dv + 1/2 (pixel i is
 *      [i, i+1)), with x_k = (v_start + k dv_bin)/dv + 1/2:
 *        Fbin_k = sum_i overlap([i, i+1), [x_k, x_{k+1})) Fc_{i mod N}
 *                 / (x_{k+1} - x_k).
 *      The n_out bins of a skewer must not exceed its box: n_out dv_bin <= V.
 *      Choosing v_start and n_out selects the observed path (for the BOSS-like
 *      spectra, the Lya-Lyb path minus 3000 km/s, clipped to the box).
 *
 *   3. Gaussian noise of standard deviation sigma (1/(S/N) in continuum units):
 *        Fobs_k = Fbin_k + sigma * eps_k,
 *      with the standard-normal draws eps supplied by the caller.
 *
 * The adjoint (oracle_instrument_backward) is the transpose of the linear map
 * F -> Fbin, written out by the chain rule: spread each bin's gradient over the
 * pixels it overlaps, then correlate with c (c is even, so this is the same
 * convolution).
 *
 * Sums use Neumaier compensation.  OpenMP over skewers only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define INS_OK 0
#define INS_EINVAL -1
#define INS_ENOMEM -5

/* Speed of light (km/s, exact) and the rest wavelengths of Lyman alpha and
 * Lyman beta (Angstrom, vacuum). */
#define INS_C_KMS 299792.458
#define INS_LYA_A 1215.67
#define INS_LYB_A 1025.72

typedef struct {
  double s, c;
} ins_acc;

static void ins_add(ins_acc *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double ins_val(const ins_acc *a) { return a->s + a->c; }

/* Velocity width of dlambda Angstrom at the Lyman-alpha line observed at
 * redshift z: dv = c dlambda / (lambda_alpha (1 + z)). */
double oracle_angstrom_to_kms(double dlambda, double z) {
  return INS_C_KMS * dlambda / (INS_LYA_A * (1.0 + z));
}

/* Velocity length of the path between a quasar's Lyman-beta and Lyman-alpha
 * lines, c ln(lambda_alpha / lambda_beta), minus the proximity zone blueward
 * of Lyman alpha (Section 3.2: 3000 km/s). */
double oracle_lya_lyb_path_kms(double proximity_kms) {
  return INS_C_KMS * log(INS_LYA_A / INS_LYB_A) - proximity_kms;
}

/* Doppler-like width of a Gaussian with the given FWHM: exp(-(d/b)^2) halves
 * at d = FWHM/2, so b = FWHM / (2 sqrt(ln 2)). */
double oracle_lsf_b(double fwhm) { return fwhm / (2.0 * sqrt(log(2.0))); }

/* Minimal image of d in [-V/2, V/2). */
static double ins_min_image(double d, double V) { return d - V * floor(d / V + 0.5); }

/* Normalised weights c_o, o = 0 .. N-1. */
static void lsf_weights(int64_t N, double dv, double fwhm, double *c) {
  if (fwhm == 0.0) {
    for (int64_t o = 0; o < N; ++o) c[o] = 0.0;
    c[0] = 1.0;
    return;
  }
  const double bL = oracle_lsf_b(fwhm);
  const double V = (double)N * dv;
  ins_acc z = {0.0, 0.0};
  for (int64_t o = 0; o < N; ++o) {
    const double d = ins_min_image((double)o * dv, V);
    c[o] = exp(-(d / bL) * (d / bL));
    ins_add(&z, c[o]);
  }
  const double Z = ins_val(&z);
  for (int64_t o = 0; o < N; ++o) c[o] /= Z;
}

/* Lower edge of bin k in pixel coordinates. */
static double bin_edge(double v_start, double bin, double dv, int64_t k) {
  return (v_start + (double)k * bin) / dv + 0.5;
}

static int64_t wrap(int64_t i, int64_t N) {
  int64_t r = i % N;
  return r < 0 ? r + N : r;
}

static int check(int64_t S, const int64_t *offsets, const double *dv, double fwhm,
                 double bin, double v_start, const int64_t *out_offsets) {
  if (S < 0 || !offsets || !dv || !out_offsets) return INS_EINVAL;
  if (!(fwhm >= 0.0) || !isfinite(fwhm) || !(bin > 0.0) || !isfinite(bin) ||
      !isfinite(v_start))
    return INS_EINVAL;
  if (offsets[0] != 0 || out_offsets[0] != 0) return INS_EINVAL;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t N = offsets[s + 1] - offsets[s];
    const int64_t n_out = out_offsets[s + 1] - out_offsets[s];
    if (N < 0 || n_out < 0) return INS_EINVAL;
    if (n_out == 0) continue;
    if (N == 0 || !(dv[s] > 0.0)) return INS_EINVAL;
    if ((double)n_out * bin > (double)N * dv[s] * (1.0 + 1e-12)) return INS_EINVAL;
  }
  return INS_OK;
}

/* Convolved spectrum of one skewer (step 1). */
static void convolve(int64_t N, const double *F, const double *c, double *Fc) {
  for (int64_t i = 0; i < N; ++i) {
    ins_acc a = {0.0, 0.0};
    for (int64_t j = 0; j < N; ++j) ins_add(&a, c[wrap(i - j, N)] * F[j]);
    Fc[i] = ins_val(&a);
  }
}

int oracle_instrument(int64_t S, const int64_t *offsets, const double *F, const double *dv,
                      double fwhm, double bin, double v_start, const int64_t *out_offsets,
                      const double *noise, double sigma, double *out) {
  int rc = check(S, offsets, dv, fwhm, bin, v_start, out_offsets);
  if (rc) return rc;
  if (!F || !out || !(sigma >= 0.0) || !isfinite(sigma) || (sigma > 0.0 && !noise))
    return INS_EINVAL;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int64_t s = 0; s < S; ++s) {
    const int64_t N = offsets[s + 1] - offsets[s];
    const int64_t n_out = out_offsets[s + 1] - out_offsets[s];
    if (n_out == 0) continue;
    double *c = (double *)malloc(sizeof(double) * (size_t)N);
    double *Fc = (double *)malloc(sizeof(double) * (size_t)N);
    if (!c || !Fc) {
      free(c);
      free(Fc);
      bad = 1;
      continue;
    }
    lsf_weights(N, dv[s], fwhm, c);
    convolve(N, F + offsets[s], c, Fc);
    for (int64_t k = 0; k < n_out; ++k) {
      const double x0 = bin_edge(v_start, bin, dv[s], k);
      const double x1 = bin_edge(v_start, bin, dv[s], k + 1);
      ins_acc a = {0.0, 0.0};
      for (int64_t i = (int64_t)floor(x0); (double)i < x1; ++i) {
        const double ov = fmin((double)(i + 1), x1) - fmax((double)i, x0);
        if (ov > 0.0) ins_add(&a, ov * Fc[wrap(i, N)]);
      }
      double v = ins_val(&a) / (x1 - x0);
      if (sigma > 0.0) v += sigma * noise[out_offsets[s] + k];
      out[out_offsets[s] + k] = v;
    }
    free(c);
    free(Fc);
  }
  return bad ? INS_ENOMEM : INS_OK;
}

/* grad_F = J^T grad_out for the linear map F -> Fbin (noise does not depend on
 * F). */
int oracle_instrument_backward(int64_t S, const int64_t *offsets, const double *dv, double fwhm,
                               double bin, double v_start, const int64_t *out_offsets,
                               const double *grad_out, double *grad_F) {
  int rc = check(S, offsets, dv, fwhm, bin, v_start, out_offsets);
  if (rc) return rc;
  if (!grad_out || !grad_F) return INS_EINVAL;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int64_t s = 0; s < S; ++s) {
    const int64_t N = offsets[s + 1] - offsets[s];
    const int64_t n_out = out_offsets[s + 1] - out_offsets[s];
    double *gF = grad_F + offsets[s];
    if (n_out == 0) {
      for (int64_t j = 0; j < N; ++j) gF[j] = 0.0;
      continue;
    }
    double *c = (double *)malloc(sizeof(double) * (size_t)N);
    ins_acc *gFc = (ins_acc *)calloc((size_t)N, sizeof(ins_acc));
    double *gc = (double *)malloc(sizeof(double) * (size_t)N);
    if (!c || !gFc || !gc) {
      free(c);
      free(gFc);
      free(gc);
      bad = 1;
      continue;
    }
    lsf_weights(N, dv[s], fwhm, c);
    /* transpose of the resampling: d Fbin_k / d Fc_i = overlap / (x1 - x0) */
    for (int64_t k = 0; k < n_out; ++k) {
      const double x0 = bin_edge(v_start, bin, dv[s], k);
      const double x1 = bin_edge(v_start, bin, dv[s], k + 1);
      const double gk = grad_out[out_offsets[s] + k] / (x1 - x0);
      for (int64_t i = (int64_t)floor(x0); (double)i < x1; ++i) {
        const double ov = fmin((double)(i + 1), x1) - fmax((double)i, x0);
        if (ov > 0.0) ins_add(&gFc[wrap(i, N)], ov * gk);
      }
    }
    for (int64_t i = 0; i < N; ++i) gc[i] = ins_val(&gFc[i]);
    /* transpose of the convolution: d Fc_i / d F_j = c_{(i-j) mod N} */
    for (int64_t j = 0; j < N; ++j) {
      ins_acc a = {0.0, 0.0};
      for (int64_t i = 0; i < N; ++i) ins_add(&a, c[wrap(i - j, N)] * gc[i]);
      gF[j] = ins_val(&a);
    }
    free(c);
    free(gFc);
    free(gc);
  }
  return bad ? INS_ENOMEM : INS_OK;
}
