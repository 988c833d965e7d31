/* oracle_sanitize.c -- drives every function of the FP64 oracle
 * (oracle/lyaf_oracle.c, oracle/lyaf_instrument_oracle.c) on small ragged
 * inputs, including empty skewers, empty pixels and invalid arguments, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  Test
 * infrastructure: it declares the oracle's prototypes itself and exits non-zero
 * on the first failed check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_tau(int64_t, const int64_t *, const double *, const double *, const double *,
               const double *, const double *, double, double, double, double *);
int oracle_tau_at(int64_t, const int64_t *, const double *, const double *, const double *,
                  const double *, const double *, double, double, int64_t, const int64_t *,
                  int64_t, double *);
int oracle_mean_flux_A(int64_t, const double *, double, double *, int *);
void oracle_finalise(int64_t, const double *, double, double *, double *);
int oracle_tau_grad(int64_t, const int64_t *, const double *, const double *, const double *,
                    const double *, const double *, double, double, const double *, double *,
                    double *, double *, double *);
int oracle_normalise_backward(int64_t, const double *, double, const double *, const double *,
                              int, double *);
int oracle_instrument(int64_t, const int64_t *, const double *, const double *, double, double,
                      double, const int64_t *, const double *, double, double *);
int oracle_instrument_backward(int64_t, const int64_t *, const double *, double, double, double,
                               const int64_t *, const double *, double *);
double oracle_min_image(double, double);

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  rng ^= rng >> 12;
  rng ^= rng << 25;
  rng ^= rng >> 27;
  return (double)((rng * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
  enum { S = 4 };
  const int64_t off[S + 1] = {0, 0, 7, 47, 111}; /* an empty skewer, then 7, 40, 64 px */
  const int64_t P = off[S];
  double *delta = malloc(sizeof(double) * P), *v = malloc(sizeof(double) * P);
  double dv[S] = {2.0, 2.0, 3.0, 1.0}, T0[S] = {1e4, 1.5e4, 2e4, 5e3},
         gm[S] = {1.5, 1.3, 0.8, 1.6};
  for (int64_t p = 0; p < P; ++p) {
    delta[p] = (p % 9 == 4) ? 0.0 : 3.0 * urand() + (p % 13 == 0 ? 20.0 : 0.0);
    v[p] = 100.0 * (urand() - 0.5);
  }
  double *full = malloc(sizeof(double) * P), *win = malloc(sizeof(double) * P);
  CHECK(oracle_tau(S, off, delta, v, dv, T0, gm, 1.0, 10.0, 0.0, full) == 0);
  CHECK(oracle_tau(S, off, delta, v, dv, T0, gm, 1.0, 10.0, 8.0, win) == 0);
  for (int64_t p = 0; p < P; ++p) CHECK(fabs(full[p] - win[p]) <= 1e-12 * (full[p] + 1e-30));
  const int64_t tg[3] = {0, 5, 39};
  double at[3];
  CHECK(oracle_tau_at(S, off, delta, v, dv, T0, gm, 1.0, 10.0, 2, tg, 3, at) == 0);
  for (int k = 0; k < 3; ++k) CHECK(at[k] == full[off[2] + tg[k]]);

  /* mean flux: uniform tau has A = -ln F / tau0 */
  double uni[17], A = 0.0;
  int it = 0;
  for (int k = 0; k < 17; ++k) uni[k] = 0.7;
  CHECK(oracle_mean_flux_A(17, uni, 0.8, &A, &it) == 0);
  CHECK(fabs(A / (-log(0.8) / 0.7) - 1.0) <= 1e-14);
  CHECK(oracle_mean_flux_A(P, full, 0.8, &A, &it) == 0);
  double *ts = malloc(sizeof(double) * P), *F = malloc(sizeof(double) * P);
  oracle_finalise(P, full, A, ts, F);
  double m = 0.0;
  for (int64_t p = 0; p < P; ++p) m += F[p];
  CHECK(fabs(m / (double)P - 0.8) <= 1e-12);

  /* adjoint */
  double *g = malloc(sizeof(double) * P), *gt = malloc(sizeof(double) * P);
  double *gd = malloc(sizeof(double) * P), *gv = malloc(sizeof(double) * P);
  double gT[S], gg[S];
  for (int64_t p = 0; p < P; ++p) g[p] = urand() - 0.5;
  CHECK(oracle_normalise_backward(P, full, A, g, NULL, 1, gt) == 0);
  CHECK(oracle_tau_grad(S, off, delta, v, dv, T0, gm, 1.0, 10.0, gt, gd, gv, gT, gg) == 0);
  for (int64_t p = 0; p < P; ++p) CHECK(isfinite(gd[p]) && isfinite(gv[p]));

  /* instrument: the adjoint satisfies <J x, y> = <x, J^T y> */
  const int64_t oo[S + 1] = {0, 0, 2, 12, 26}; /* every bin run shorter than its box */
  double *x = malloc(sizeof(double) * P), *y = malloc(sizeof(double) * oo[S]);
  double *Jx = malloc(sizeof(double) * oo[S]), *Jty = malloc(sizeof(double) * P);
  for (int64_t p = 0; p < P; ++p) x[p] = urand();
  for (int64_t k = 0; k < oo[S]; ++k) y[k] = urand() - 0.5;
  CHECK(oracle_instrument(S, off, x, dv, 7.0, 4.5, 1.0, oo, NULL, 0.0, Jx) == 0);
  CHECK(oracle_instrument_backward(S, off, dv, 7.0, 4.5, 1.0, oo, y, Jty) == 0);
  double l = 0.0, r = 0.0;
  for (int64_t k = 0; k < oo[S]; ++k) l += Jx[k] * y[k];
  for (int64_t p = 0; p < P; ++p) r += x[p] * Jty[p];
  CHECK(fabs(l - r) <= 1e-12 * (fabs(l) + 1.0));

  /* invalid arguments are rejected */
  CHECK(oracle_tau(-1, off, delta, v, dv, T0, gm, 1.0, 10.0, 0.0, full) != 0);
  CHECK(oracle_tau(S, NULL, delta, v, dv, T0, gm, 1.0, 10.0, 0.0, full) != 0);
  CHECK(oracle_mean_flux_A(0, uni, 0.8, &A, &it) != 0);
  CHECK(oracle_mean_flux_A(17, uni, 1.5, &A, &it) != 0);
  CHECK(oracle_normalise_backward(P, NULL, A, g, NULL, 1, gt) != 0);
  CHECK(oracle_min_image(3.0, 4.0) == -1.0);

  free(delta); free(v); free(full); free(win); free(ts); free(F); free(g); free(gt);
  free(gd); free(gv); free(x); free(y); free(Jx); free(Jty);
  puts("oracle_sanitize: ok");
  return 0;
}
