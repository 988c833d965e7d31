/*
 * lyaf_oracle.c -- plain FP64 CPU oracle for the Lyman-alpha optical-depth path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no header, constant or helper with the HIP
 * library: every physical constant and every formula below is written out again
 * here, from the paper (Greig, Bolton & Wyithe 2011, Section 2.3).
 *
 * What it computes, in IEEE double precision, round-to-nearest, no fast-math:
 *
 *   Temperature-density relation with pivot (Sec. 2.3, eq. 5 and the text that
 *   follows it): D_j = Delta_j if Delta_j <= Delta_p, else Delta_p;
 *   T_j = T0 * D_j^(gamma-1).
 *
 *   Doppler parameter (Sec. 2.3, after eq. 6): b_j = sqrt(2 k_B T_j / m_H).
 *
 *   Neutral density in photo-ionisation equilibrium (Sec. 2.3, eq. 4):
 *   n_HI(j) proportional to Delta_j^2 (T_j / 1e4 K)^-0.7.  Every constant factor
 *   of eq. (4) and of the prefactor c sigma_alpha deltaR / sqrt(pi) of eq. (6)
 *   is folded into one number tau_ref: the optical depth of a uniform field at
 *   Delta = 1 and T = 1e4 K.  With pixel width dv = H deltaR (km/s) the weight of
 *   source j is  w_j = tau_ref Delta_j^2 (T_j/1e4)^-0.7 dv / (sqrt(pi) b_j).
 *
 *   Optical depth (Sec. 2.3, eq. 6), full O(N^2) sum, periodic box of width
 *   V = N dv in velocity space, each source taken at its minimal image:
 *   tau_i = sum_j w_j exp(-(d_ij / b_j)^2),
 *   d_ij = (i - j) dv - v_j, reduced to [-V/2, V/2).
 *   Here v_j is the peculiar velocity; v_H(i) - u(j) = (i - j) dv - v_pec(j)
 *   because u(j) = v_H(j) + v_pec(j) and v_H(i) - v_H(j) = (i - j) dv.
 *   A source with Delta_j = 0 contributes exactly 0 (the limit of eq. 4).
 *
 *   Mean-flux normalisation (Sec. 2.3, last paragraph): the constant A solves
 *   (1/P) sum_p exp(-A tau_p) = Fbar over all pixels of all skewers; then
 *   tau' = A tau and F = exp(-tau').
 *
 *   Gradient of a scalar loss through eqs. (4)-(6) and through A (implicit
 *   differentiation of the normalisation condition), written out from the chain
 *   rule; see oracle_tau_grad and oracle_normalise_backward.
 *
 * Sums use Neumaier (improved Kahan-Babuska) compensation.  Skewers are
 * independent, so an OpenMP loop over skewers is the only parallelism; the
 * arithmetic inside each skewer is sequential and in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CGS constants (CODATA 2018 exact k_B; m_H = mass of the hydrogen atom). */
#define ORC_KBOLTZ 1.380649e-16   /* erg / K */
#define ORC_MHYDROGEN 1.6735575e-24 /* g */
#define ORC_CM_PER_KM 1.0e5

/* Error codes returned by the oracle entry points. */
#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EDOMAIN -2
#define ORC_ENOROOT -3
#define ORC_ENOCONV -4

/* ------------------------------------------------------------------------- */
/* Neumaier compensated accumulator.                                          */
typedef struct { double s, c; } orc_acc;

static void acc_add(orc_acc *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double acc_val(const orc_acc *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------- */
/* Doppler parameter b = sqrt(2 k_B T / m_H), in km/s (Sec. 2.3, after eq. 6). */
double oracle_doppler_b(double T) {
  return sqrt(2.0 * ORC_KBOLTZ * T / ORC_MHYDROGEN) / ORC_CM_PER_KM;
}

/* Per-source quantities of one pixel (Sec. 2.3, eqs. 4-5).
 * Outputs: D (density entering the T-rho relation), T, b, w. */
typedef struct { double D, T, b, w; } orc_src;

static orc_src source_params(double delta, double dv, double T0, double gamma,
                             double tau_ref, double delta_pivot) {
  orc_src s;
  if (delta == 0.0) { /* empty pixel: no neutral hydrogen, no line */
    s.D = 0.0; s.T = 0.0; s.b = 0.0; s.w = 0.0;
    return s;
  }
  /* eq. (5) below the pivot; constant temperature above it */
  s.D = (delta <= delta_pivot) ? delta : delta_pivot;
  s.T = T0 * pow(s.D, gamma - 1.0);
  s.b = oracle_doppler_b(s.T);
  /* eq. (4) shape times the eq. (6) prefactor, normalised by tau_ref */
  s.w = tau_ref * delta * delta * pow(s.T / 1.0e4, -0.7) * dv /
        (sqrt(M_PI) * s.b);
  return s;
}

/* Exported for tests: the four per-source quantities of one pixel. */
void oracle_source_params(double delta, double dv, double T0, double gamma,
                          double tau_ref, double delta_pivot, double *D,
                          double *T, double *b, double *w) {
  orc_src s = source_params(delta, dv, T0, gamma, tau_ref, delta_pivot);
  *D = s.D; *T = s.T; *b = s.b; *w = s.w;
}

/* Minimal periodic image of a velocity offset: reduce d to [-V/2, V/2). */
double oracle_min_image(double d, double V) {
  return d - V * floor((d + 0.5 * V) / V);
}

/* ------------------------------------------------------------------------- */
static int check_skewers(int64_t n_skewers, const int64_t *offsets,
                         const double *delta, const double *vpec,
                         const double *dv, const double *T0,
                         const double *gamma, double tau_ref,
                         double delta_pivot) {
  if (n_skewers < 0 || !offsets) return ORC_EINVAL;
  if (offsets[0] != 0) return ORC_EINVAL;
  for (int64_t s = 0; s < n_skewers; ++s)
    if (offsets[s + 1] < offsets[s]) return ORC_EINVAL;
  if (!(tau_ref > 0.0) || !(delta_pivot > 0.0)) return ORC_EINVAL;
  for (int64_t s = 0; s < n_skewers; ++s) {
    if (!(dv[s] > 0.0) || !isfinite(dv[s])) return ORC_EDOMAIN;
    if (!(T0[s] > 0.0) || !isfinite(T0[s])) return ORC_EDOMAIN;
    if (!isfinite(gamma[s])) return ORC_EDOMAIN;
  }
  int64_t P = offsets[n_skewers];
  for (int64_t p = 0; p < P; ++p) {
    if (!(delta[p] >= 0.0) || !isfinite(delta[p])) return ORC_EDOMAIN;
    if (!isfinite(vpec[p])) return ORC_EDOMAIN;
  }
  return ORC_OK;
}

/* Optical depth, eq. (6), every skewer, every pixel.
 *   window_k == 0: the full sum over all sources (the definition).
 *   window_k  > 0: only sources with |d_ij| < window_k * b_j enter the sum; the
 *                  terms left out are each below exp(-window_k^2) of their
 *                  source's peak.  Used only to time the oracle on large
 *                  samples; tests compare it with the full sum.
 * Layout: skewer s owns pixels offsets[s] .. offsets[s+1]-1 of every [P] array. */
int oracle_tau(int64_t n_skewers, const int64_t *offsets, const double *delta,
               const double *vpec, const double *dv, const double *T0,
               const double *gamma, double tau_ref, double delta_pivot,
               double window_k, double *tau_out) {
  int rc = check_skewers(n_skewers, offsets, delta, vpec, dv, T0, gamma,
                         tau_ref, delta_pivot);
  if (rc) return rc;
  if (!(window_k >= 0.0)) return ORC_EINVAL;

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < n_skewers; ++s) {
    const int64_t off = offsets[s];
    const int64_t N = offsets[s + 1] - off;
    if (N == 0) continue;
    const double V = (double)N * dv[s];
    orc_src *src = (orc_src *)malloc((size_t)N * sizeof(orc_src));
    for (int64_t j = 0; j < N; ++j)
      src[j] = source_params(delta[off + j], dv[s], T0[s], gamma[s], tau_ref,
                             delta_pivot);
    for (int64_t i = 0; i < N; ++i) {
      orc_acc acc = {0.0, 0.0};
      for (int64_t j = 0; j < N; ++j) {
        if (src[j].w == 0.0) continue;
        double d = oracle_min_image((double)(i - j) * dv[s] - vpec[off + j], V);
        if (window_k > 0.0 && !(fabs(d) < window_k * src[j].b)) continue;
        double x = d / src[j].b;
        acc_add(&acc, src[j].w * exp(-x * x));
      }
      tau_out[off + i] = acc_val(&acc);
    }
    free(src);
  }
  return ORC_OK;
}

/* Optical depth, eq. (6), at chosen pixels of one skewer: the full sum of
 * oracle_tau with window_k = 0 (same terms, same order), for skewers too long
 * for an all-pixel O(N^2) pass.  tau_out[t] = tau of pixel targets[t]
 * (0 <= targets[t] < N) of skewer s; the targets are spread over threads. */
int oracle_tau_at(int64_t n_skewers, const int64_t *offsets, const double *delta,
                  const double *vpec, const double *dv, const double *T0,
                  const double *gamma, double tau_ref, double delta_pivot,
                  int64_t s, const int64_t *targets, int64_t n_targets,
                  double *tau_out) {
  int rc = check_skewers(n_skewers, offsets, delta, vpec, dv, T0, gamma,
                         tau_ref, delta_pivot);
  if (rc) return rc;
  if (s < 0 || s >= n_skewers || n_targets < 0) return ORC_EINVAL;
  const int64_t off = offsets[s];
  const int64_t N = offsets[s + 1] - off;
  for (int64_t t = 0; t < n_targets; ++t)
    if (targets[t] < 0 || targets[t] >= N) return ORC_EINVAL;
  const double V = (double)N * dv[s];
  orc_src *src = (orc_src *)malloc((size_t)(N > 0 ? N : 1) * sizeof(orc_src));
  if (!src) return ORC_EINVAL;
  for (int64_t j = 0; j < N; ++j)
    src[j] = source_params(delta[off + j], dv[s], T0[s], gamma[s], tau_ref,
                           delta_pivot);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < n_targets; ++t) {
    const int64_t i = targets[t];
    orc_acc acc = {0.0, 0.0};
    for (int64_t j = 0; j < N; ++j) {
      if (src[j].w == 0.0) continue;
      double d = oracle_min_image((double)(i - j) * dv[s] - vpec[off + j], V);
      double x = d / src[j].b;
      acc_add(&acc, src[j].w * exp(-x * x));
    }
    tau_out[t] = acc_val(&acc);
  }
  free(src);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Mean-flux normalisation (Sec. 2.3, last paragraph).
 * g(A) = (1/P) sum_p exp(-A tau_p) - Fbar is strictly decreasing in A when some
 * tau_p > 0, with g(0) = 1 - Fbar and g(inf) = z0 - Fbar, z0 the fraction of
 * pixels with tau_p = 0.  A root exists iff z0 < Fbar < 1.
 * Method: bracket [lo, hi] with g(lo) > 0 > g(hi), found by doubling hi, then
 * Newton steps that fall back to bisection whenever they leave the bracket,
 * until the step is below 1e-15 of A.  Outputs A and the iteration count. */
static void flux_sums(int64_t P, const double *tau, double A, double *g0,
                      double *g1) {
  orc_acc s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
  for (int64_t p = 0; p < P; ++p) {
    double e = exp(-A * tau[p]);
    acc_add(&s0, e);
    acc_add(&s1, tau[p] * e);
  }
  *g0 = acc_val(&s0);
  *g1 = acc_val(&s1);
}

int oracle_mean_flux_A(int64_t P, const double *tau, double target_F,
                       double *A_out, int *n_iter) {
  if (P <= 0 || !tau || !A_out) return ORC_EINVAL;
  if (!(target_F > 0.0 && target_F < 1.0)) return ORC_EINVAL;
  int64_t n_zero = 0;
  orc_acc tsum = {0.0, 0.0};
  for (int64_t p = 0; p < P; ++p) {
    if (!(tau[p] >= 0.0) || !isfinite(tau[p])) return ORC_EDOMAIN;
    if (tau[p] == 0.0) ++n_zero;
    acc_add(&tsum, tau[p]);
  }
  const double Pd = (double)P;
  if (!((double)n_zero / Pd < target_F)) return ORC_ENOROOT;
  const double mean_tau = acc_val(&tsum) / Pd;

  double lo = 0.0, hi = 1.0 / mean_tau, s0, s1;
  int it = 0;
  for (;;) { /* grow the bracket until g(hi) < 0 */
    flux_sums(P, tau, hi, &s0, &s1);
    if (s0 / Pd - target_F < 0.0) break;
    lo = hi;
    hi *= 2.0;
    if (++it > 2000) return ORC_ENOCONV;
  }
  double A = 0.5 * (lo + hi);
  for (int k = 0; k < 500; ++k, ++it) {
    flux_sums(P, tau, A, &s0, &s1);
    const double g = s0 / Pd - target_F;
    const double dg = -s1 / Pd;
    if (g == 0.0) { /* A is a root to the precision of the sums */
      *A_out = A;
      if (n_iter) *n_iter = it + 1;
      return ORC_OK;
    }
    if (g > 0.0) lo = A; else hi = A;
    double An = (dg < 0.0) ? A - g / dg : 0.5 * (lo + hi);
    if (!(An > lo && An < hi)) An = 0.5 * (lo + hi);
    if (fabs(An - A) <= 1e-15 * A) {
      *A_out = An;
      if (n_iter) *n_iter = it + 1;
      return ORC_OK;
    }
    A = An;
  }
  return ORC_ENOCONV;
}

/* tau' = A tau and F = exp(-tau') (Sec. 2.3: F = exp(-tau) after rescaling). */
void oracle_finalise(int64_t P, const double *tau, double A, double *tau_out,
                     double *F_out) {
  for (int64_t p = 0; p < P; ++p) {
    const double t = A * tau[p];
    if (tau_out) tau_out[p] = t;
    if (F_out) F_out[p] = exp(-t);
  }
}

/* ------------------------------------------------------------------------- */
/* Gradient of a loss L through eq. (6) with eqs. (4)-(5) (chain rule).
 * Input g[P] = dL/dtau_i (raw optical depth, before the mean-flux rescale).
 * For each source j, with x = d_ij / b_j and E = exp(-x^2):
 *   S0_j = sum_i g_i w_j E,  S1_j = sum_i g_i w_j E x,  S2_j = sum_i g_i w_j E x^2.
 *   dtau_i/dv_j   = w_j E 2x / b_j                 -> dL/dv_j = 2 S1_j / b_j
 *   dtau_i/dlnT_j = w_j E (x^2 - 1.2)              -> Q_j = S2_j - 1.2 S0_j
 *     (w ~ T^-0.7 / b ~ T^-1.2; x^2 ~ 1/T)
 *   dlnT_j/dlnDelta_j = (gamma - 1) below the pivot, 0 above it (eq. 5)
 *   dL/dDelta_j = [2 S0_j + (gamma-1) [Delta_j <= Delta_p] Q_j] / Delta_j
 *   dL/dT0      = sum_j Q_j / T0,   dL/dgamma = sum_j Q_j ln D_j   (per skewer)
 * A source with Delta_j = 0 has w_j = 0 and gets gradient 0. */
int oracle_tau_grad(int64_t n_skewers, const int64_t *offsets,
                    const double *delta, const double *vpec, const double *dv,
                    const double *T0, const double *gamma, double tau_ref,
                    double delta_pivot, const double *g, double *grad_delta,
                    double *grad_vpec, double *grad_T0, double *grad_gamma) {
  int rc = check_skewers(n_skewers, offsets, delta, vpec, dv, T0, gamma,
                         tau_ref, delta_pivot);
  if (rc) return rc;

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < n_skewers; ++s) {
    const int64_t off = offsets[s];
    const int64_t N = offsets[s + 1] - off;
    orc_acc gT0 = {0.0, 0.0}, ggam = {0.0, 0.0};
    const double V = (double)N * dv[s];
    for (int64_t j = 0; j < N; ++j) {
      orc_src sj = source_params(delta[off + j], dv[s], T0[s], gamma[s],
                                 tau_ref, delta_pivot);
      if (sj.w == 0.0) {
        grad_delta[off + j] = 0.0;
        grad_vpec[off + j] = 0.0;
        continue;
      }
      orc_acc S0 = {0.0, 0.0}, S1 = {0.0, 0.0}, S2 = {0.0, 0.0};
      for (int64_t i = 0; i < N; ++i) {
        double d = oracle_min_image((double)(i - j) * dv[s] - vpec[off + j], V);
        double x = d / sj.b;
        double t = g[off + i] * sj.w * exp(-x * x);
        acc_add(&S0, t);
        acc_add(&S1, t * x);
        acc_add(&S2, t * x * x);
      }
      const double s0 = acc_val(&S0), s1 = acc_val(&S1), s2 = acc_val(&S2);
      const double Q = s2 - 1.2 * s0;
      const double below = (delta[off + j] <= delta_pivot) ? 1.0 : 0.0;
      grad_vpec[off + j] = 2.0 * s1 / sj.b;
      grad_delta[off + j] =
          (2.0 * s0 + (gamma[s] - 1.0) * below * Q) / delta[off + j];
      acc_add(&gT0, Q / T0[s]);
      acc_add(&ggam, Q * log(sj.D));
    }
    grad_T0[s] = acc_val(&gT0);
    grad_gamma[s] = acc_val(&ggam);
  }
  return ORC_OK;
}

/* Backward of the mean-flux normalisation.
 * Forward: A(tau) solves sum_p exp(-A tau_p) = P Fbar; tau'_p = A tau_p;
 * F_p = exp(-tau'_p).  Given dL/dF (grad_F) and dL/dtau' (grad_tau_scaled),
 * either may be NULL (zero), with G_p = dL/dtau'_p - F_p dL/dF_p:
 *   frozen A   : dL/dtau_p = A G_p
 *   implicit A : differentiating the constraint gives
 *                dA = -A sum_p F_p dtau_p / sum_p F_p tau_p, hence
 *                dL/dtau_p = A G_p - A F_p (sum_q G_q tau_q) / (sum_q F_q tau_q).
 * Output: grad_tau_raw[P] = dL/dtau_p. */
int oracle_normalise_backward(int64_t P, const double *tau_raw, double A,
                              const double *grad_F,
                              const double *grad_tau_scaled, int implicit_A,
                              double *grad_tau_raw) {
  if (P < 0 || !tau_raw || !grad_tau_raw) return ORC_EINVAL;
  double *G = (double *)malloc((size_t)(P > 0 ? P : 1) * sizeof(double));
  double *F = (double *)malloc((size_t)(P > 0 ? P : 1) * sizeof(double));
  orc_acc sGt = {0.0, 0.0}, sFt = {0.0, 0.0};
  for (int64_t p = 0; p < P; ++p) {
    F[p] = exp(-A * tau_raw[p]);
    G[p] = (grad_tau_scaled ? grad_tau_scaled[p] : 0.0) -
           F[p] * (grad_F ? grad_F[p] : 0.0);
    acc_add(&sGt, G[p] * tau_raw[p]);
    acc_add(&sFt, F[p] * tau_raw[p]);
  }
  const double ratio =
      (implicit_A && acc_val(&sFt) != 0.0) ? acc_val(&sGt) / acc_val(&sFt) : 0.0;
  for (int64_t p = 0; p < P; ++p)
    grad_tau_raw[p] = A * G[p] - (implicit_A ? A * F[p] * ratio : 0.0);
  free(G);
  free(F);
  return ORC_OK;
}

/* Number of threads the OpenMP loops use (reported next to oracle timings). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
