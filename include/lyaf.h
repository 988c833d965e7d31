/*
 * lyaf.h -- C ABI of the MI355X (gfx950) Lyman-alpha optical-depth library.
 *
 * The library computes, for a batch of sight-lines ("skewers") of gridded
 * overdensity Delta and peculiar velocity v, the Lyman-alpha optical depth of
 * Greig, Bolton & Wyithe (2011), Section 2.3:
 *
 *   T_j   = T0 * D_j^(gamma-1),  D_j = min(Delta_j, delta_pivot)   (eq. 5 + pivot)
 *   b_j   = sqrt(2 k_B T_j / m_H)                                  (after eq. 6)
 *   w_j   = tau_ref * Delta_j^2 * (T_j / 1e4 K)^-0.7 * dv / (sqrt(pi) b_j)
 *                                                    (eq. 4 inside eq. 6)
 *   tau_i = sum_j w_j * exp(-(d_ij / b_j)^2),  d_ij = (i - j) dv - v_j   (eq. 6)
 *
 * with d_ij taken at its minimal periodic image in a box of width V = N dv, and
 * then the mean-flux renormalisation of Section 2.3: A solves
 * (1/P) sum_p exp(-A tau_p) = target_F over every pixel of every skewer,
 * tau' = A tau and F = exp(-tau').
 *
 * tau_ref folds every constant of eq. (4) and the prefactor c sigma_alpha
 * deltaR / sqrt(pi) of eq. (6): it is the optical depth of a uniform field at
 * Delta = 1 and T = 1e4 K.  Because the mean-flux rescale absorbs any constant
 * factor, tau_ref only sets the scale of the raw tau.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers marked DEVICE point to memory of the current HIP device, owned by
 *   the caller (for example torch tensors).  Pointers marked HOST point to host
 *   memory read during the call only.  The library never frees, reallocates or
 *   keeps caller memory.
 * - Layout: skewer s owns pixels offsets[s] .. offsets[s+1]-1 of every [P]
 *   array (skewer-major, pixel fastest, contiguous).
 * - `stream` is a hipStream_t passed as void*; NULL is the null stream.  All
 *   work is enqueued on it; no call synchronises the host unless stated.
 * - Return value: LYAF_OK (0) or a negative LYAF_E* code.  Every error a host
 *   can see (null pointers, bad sizes or offsets, bad parameters) is reported
 *   before anything is enqueued, and the outputs are then untouched.
 * - Data errors that only the device can see (Delta < 0 or non-finite, v
 *   non-finite, dv <= 0, T0 <= 0, gamma non-finite, tau < 0, no mean-flux
 *   root) set bits in a sticky per-device status word (LYAF_STATUS_*), read
 *   and cleared by lyaf_status_read.  Outputs are unspecified when it is set.
 * - Outputs are overwritten, never accumulated into.
 * - The library keeps per-device, per-stream workspaces (a few MB at most),
 *   allocated on the first call that needs them and reused afterwards; calls
 *   that overlap on one stream are ordered by the stream, calls on different
 *   streams do not share workspace.
 */
#ifndef LYAF_H
#define LYAF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define LYAF_OK 0
#define LYAF_EINVAL -1   /* bad argument detected on the host */
#define LYAF_EDOMAIN -2  /* value outside the model's domain (host-visible) */
#define LYAF_ENOROOT -3  /* no mean-flux root exists */
#define LYAF_ENOCONV -4  /* root-find did not converge */
#define LYAF_EDEVICE -5  /* a HIP runtime call failed */
#define LYAF_ENOMEM -6   /* device allocation failed */

/* ---- device status bits (lyaf_status_read) ---- */
#define LYAF_STATUS_DOMAIN 1u  /* Delta<0, NaN/Inf input, dv<=0, T0<=0, tau<0 */
#define LYAF_STATUS_NOROOT 2u  /* fraction of tau == 0 pixels >= target_F */
#define LYAF_STATUS_NOCONV 4u  /* mean-flux iteration hit its cap */

/* ---- lyaf_params.flags ---- */
/* Plain form: the full O(N^2) sum of eq. (6), one thread per pixel, naive
 * FP32 accumulation, one launch per skewer.  The comparison baseline. */
#define LYAF_FLAG_PLAIN 1u
/* Launch the windowed kernel once per skewer instead of one batched launch. */
#define LYAF_FLAG_PER_SKEWER 2u
/* Persistent work-queue launch of the windowed kernel (see plans below). */
#define LYAF_FLAG_PERSISTENT 4u
/* Force windowed-kernel shape v (0 .. LYAF_NUM_SHAPES-1; the shapes a plan's
 * tuner chooses from): flags |= LYAF_FLAG_SHAPE(v); without the flag (and in
 * a plan created without LYAF_PLAN_AUTOTUNE) shape 4 runs.  0: each lane owns
 * 4 consecutive targets and walks its own run of sources, one source stream
 * per wave, 1024-pixel tiles; 1: the same with 512-pixel tiles;
 * 2: 8 source streams share 32-target sub-tiles, 4 targets per lane,
 * 512-pixel tiles; 3: as 2 with 2 targets per lane; 4: as 0 with the
 * Gaussian of a source evaluated across the lane's 4 targets by a product
 * recurrence (two exp2 per source and lane instead of four; a tile holding a
 * line narrower than sqrt(log2 e) pixel widths, b < 1.2 dv, falls back to
 * shape 0's arithmetic); 5: the recurrence over 8 targets per lane, 2048-pixel
 * tiles (two exp2 per eight pairs; fallback below b = 2.7 dv, and tiles whose
 * reach exceeds 200 pixels take the full-sum path). */
#define LYAF_NUM_SHAPES 6
#define LYAF_FLAG_SHAPE(v) ((((uint32_t)(v)) + 1u) << 8)

typedef struct lyaf_skewers {
  int64_t n_skewers;      /* S >= 0 */
  const int64_t *offsets; /* HOST [S+1]: offsets[0] = 0, non-decreasing; P = offsets[S] */
  const float *delta;     /* DEVICE [P]: Delta = 1 + delta_b >= 0 (0: empty pixel, no line) */
  const float *vpec;      /* DEVICE [P]: peculiar velocity along the line of sight, km/s */
  const float *dv;        /* DEVICE [S]: pixel width in velocity, km/s (> 0) */
  const float *T0;        /* DEVICE [S]: temperature at mean density, K (> 0) */
  const float *gamma;     /* DEVICE [S]: slope of the T-rho relation (finite; < 1 allowed) */
} lyaf_skewers;

typedef struct lyaf_params {
  double tau_ref;     /* > 0: optical depth of Delta = 1, T = 1e4 K gas */
  double delta_pivot; /* > 0: T is held at T(delta_pivot) above it (10 in the paper); +INF disables */
  double window_k;    /* >= 0: sum only |d| < window_k * b (6 is exact to exp(-36) per term);
                         0 = full sum over every source */
  uint32_t flags;     /* LYAF_FLAG_* */
} lyaf_params;

/* Raw optical depth, eq. (6) with eqs. (4)-(5), for every pixel of every
 * skewer (Section 2.3).  FP32 arithmetic with compensated accumulation.
 *   tau_out: DEVICE [P] float, written.
 * Errors: EINVAL (null pointer with P > 0, S < 0, bad offsets, tau_ref <= 0,
 * delta_pivot <= 0, window_k < 0 or non-finite), EDEVICE, ENOMEM. */
int lyaf_tau(const lyaf_skewers *sk, const lyaf_params *prm, float *tau_out,
             void *stream);

/* Mean-flux renormalisation (Section 2.3, last paragraph): solve
 * (1/P) sum_p exp(-A tau_p) = target_F for A in FP64 on the device (from the
 * root on a sample of the pixels, a step to the root of the series of the
 * mean flux about it, with safeguarded Newton/Halley steps as the fallback;
 * FP64 sums), then write tau' = A tau and F = exp(-tau').
 *   tau_inout: DEVICE [n_pix] float; raw tau in, A*tau out (may not alias F_out).
 *   F_out:     DEVICE [n_pix] float, written (may be NULL to skip).
 *   A_dev:     DEVICE double, written with A.
 * No host synchronisation: a missing root or a non-converged iteration is
 * reported through the status word (A is then left at its last iterate).
 * Errors: EINVAL (n_pix <= 0 or > 2^48, null pointers, target_F not in (0, 1)),
 * EDEVICE, ENOMEM. */
int lyaf_normalise_mean_flux(int64_t n_pix, float *tau_inout, float *F_out,
                             double target_F, double *A_dev, void *stream);

/* Allocation-free lyaf_normalise_mean_flux, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as
 * lyaf_normalise_mean_flux (bitwise-identical tau' and F), plus:
 *   status_dev: DEVICE uint32 or NULL; LYAF_STATUS_* bits of this call are
 *               OR'd into it (the caller clears it).  NULL discards them.
 * It calls no hipMalloc, hipFree or other allocating routine and takes no
 * library lock: its scratch (partial sums, the root-find sample and states,
 * LYAF_NORM_NOALLOC_SCRATCH_BYTES per device) is one static device array that
 * every call on that device shares, set up on the first call on the device.
 * Calls that overlap in time on one device (different streams or threads)
 * therefore race and give wrong results; serialise them.  Any n_pix up to
 * 2^48 fits the fixed scratch (larger sizes: EINVAL). */
#define LYAF_NORM_NOALLOC_SCRATCH_BYTES 131840
int lyaf_normalise_mean_flux_noalloc(int64_t n_pix, float *tau_inout, float *F_out,
                                     double target_F, double *A_dev, uint32_t *status_dev,
                                     void *stream);

/* Backward of lyaf_normalise_mean_flux.  With G_p = dL/dtau'_p - F_p dL/dF_p:
 *   implicit_A = 0: dL/dtau_p = A G_p (A held fixed)
 *   implicit_A = 1: A re-solved at fixed mean flux (implicit differentiation):
 *     dL/dtau_p = A G_p - A F_p (sum_q G_q tau_q) / (sum_q F_q tau_q)
 *   tau_raw: DEVICE [n_pix] raw tau (before the rescale); A_dev: DEVICE double.
 *   grad_F, grad_tau_scaled: DEVICE [n_pix] or NULL (= zero).
 *   grad_tau_raw_out: DEVICE [n_pix], written.
 * Errors: EINVAL, EDEVICE, ENOMEM. */
int lyaf_normalise_mean_flux_backward(int64_t n_pix, const float *tau_raw,
                                      const double *A_dev, const float *grad_F,
                                      const float *grad_tau_scaled,
                                      int implicit_A, float *grad_tau_raw_out,
                                      void *stream);

/* Adjoint of lyaf_tau (chain rule through eqs. 4-6).  For each source j, with
 * x = d_ij / b_j and E = exp(-x^2), S0_j = sum_i g_i w_j E, S1_j = sum_i g_i w_j E x,
 * S2_j = sum_i g_i w_j E x^2, Q_j = S2_j - 1.2 S0_j:
 *   dL/dv_j     = 2 S1_j / b_j
 *   dL/dDelta_j = [2 S0_j + (gamma - 1) [Delta_j <= delta_pivot] Q_j] / Delta_j
 *   dL/dT0_s    = sum_{j in s} Q_j / T0_s
 *   dL/dgamma_s = sum_{j in s} Q_j ln D_j
 * (Delta_j = 0 gives 0.)  The same window as lyaf_tau is used.
 *   grad_tau_raw: DEVICE [P] float (dL/dtau_raw).
 *   grad_delta, grad_vpec: DEVICE [P] float, written.
 *   grad_T0, grad_gamma: DEVICE [S] double, written (either may be NULL).
 * Errors: as lyaf_tau. */
int lyaf_tau_backward(const lyaf_skewers *sk, const lyaf_params *prm,
                      const float *grad_tau_raw, float *grad_delta,
                      float *grad_vpec, double *grad_T0, double *grad_gamma,
                      void *stream);

/* ---- instrument model: mock observations of the flux ----
 *
 * Sections 3.1, 3.2 and 4.2 turn each flux spectrum into a mock observation:
 * convolution with a Gaussian line-spread function of given FWHM, resampling
 * onto coarser bins, and Gaussian noise of given S/N (the BOSS-like spectra of
 * Section 3.2 are also restricted to the quasar's Lya-Lyb path minus 3000 km/s,
 * which lyaf_lya_lyb_path_kms gives).  For skewer s of N pixels of width dv:
 *
 *   Fc_i   = sum_m c_m F_{(i-m) mod N},  c_m = g(m dv) / sum_m' g(m' dv),
 *            g(d) = exp(-(d / b_L)^2),  b_L = FWHM / (2 sqrt(ln 2)),
 *            over the taps |m dv| <= window_k b_L (the whole box at minimal
 *            images when that reaches half the box or window_k = 0);
 *   Fbin_k = average over [v_start + k bin, v_start + (k+1) bin) (periodic) of
 *            the spectrum that is constant, Fc_i, on pixel i, which covers
 *            velocities [(i - 1/2) dv, (i + 1/2) dv);
 *   Fobs_k = Fbin_k + noise_sigma * noise_k.
 *
 * The truncation error of the taps is below exp(-window_k^2) of the total
 * weight (6 gives 2.3e-16).  FWHM = 0 skips the convolution. */
typedef struct {
  double fwhm_kms;     /* FWHM of the line-spread function, km/s, finite, >= 0 */
  double bin_kms;      /* width of an output bin, km/s, finite, > 0 */
  double v_start_kms;  /* lower edge of every skewer's first bin, km/s, finite */
  double noise_sigma;  /* noise standard deviation (1/(S/N) in continuum units), >= 0 */
  double window_k;     /* tap truncation in units of b_L, >= 0; 0 = whole box */
} lyaf_instrument_params;

/* Mock observation of a batch of flux skewers.
 *   offsets:     HOST [S+1] int64 pixel offsets, as in lyaf_skewers.
 *   dv:          DEVICE [S] float pixel widths, km/s (> 0).
 *   F:           DEVICE [P] float flux.
 *   out_offsets: HOST [S+1] int64: skewer s yields out_offsets[s+1] -
 *                out_offsets[s] bins (0 allowed), written to F_obs from
 *                out_offsets[s].  A skewer with bins needs N > 0 pixels.
 *   noise:       DEVICE [P_out] float standard-normal draws, read only when
 *                noise_sigma > 0 (then required); the caller draws them.
 *   F_obs:       DEVICE [P_out] float, written.
 * Host-visible errors (EINVAL): NULL pointers, bad offsets, parameters out of
 * range.  Device-visible (LYAF_STATUS_DOMAIN, skewer skipped): dv <= 0 or not
 * finite, bins longer than the box (n_out bin > N dv), or a bin wider than 252
 * pixels. */
int lyaf_instrument(int64_t n_skewers, const int64_t *offsets, const float *dv, const float *F,
                    const lyaf_instrument_params *ip, const int64_t *out_offsets,
                    const float *noise, float *F_obs, void *stream);

/* Adjoint of lyaf_instrument: grad_F = J^T grad_obs for the linear map
 * F -> Fbin (the noise does not depend on F).  grad_obs: DEVICE [P_out] float;
 * grad_F: DEVICE [P] float, written (zero for skewers without bins).  Same
 * arguments and errors as lyaf_instrument (noise_sigma is ignored). */
int lyaf_instrument_backward(int64_t n_skewers, const int64_t *offsets, const float *dv,
                             const lyaf_instrument_params *ip, const int64_t *out_offsets,
                             const float *grad_obs, float *grad_F, void *stream);

/* Velocity width of dlambda Angstrom at Lyman alpha observed at redshift z:
 * c dlambda / (1215.67 A (1 + z)).  At z = 3, 3.63 A is 223.8 km/s (Section
 * 3.2 prints ~224). */
double lyaf_angstrom_to_kms(double dlambda_angstrom, double z);
/* Velocity length of a quasar's Lya-Lyb path, c ln(1215.67 / 1025.72), minus
 * the proximity zone (Section 3.2: 3000 km/s). */
double lyaf_lya_lyb_path_kms(double proximity_kms);

/* ---- flux statistics (Section 4) ----
 *
 * Flux PDF (Section 4.2): 21 bins of width 0.05 centred on F = 0, 0.05, .., 1;
 * bin j holds 0.05 j - 0.025 <= F < 0.05 j + 0.025, decided as
 * j = floor((F + 0.025) * 20) in IEEE double on the exact float input.
 *   F:      DEVICE [n_pix] float (any flux, e.g. F or the instrument's F_obs).
 *   counts: DEVICE [24] int64, written: bins 0..20, then the number below the
 *           first bin, at or above the end of the last, and NaN.  Exact.
 * Errors: EINVAL for n_pix < 0 or NULL pointers (F may be NULL when n_pix = 0).
 * The normalised PDF is counts[j] / (sum of counts[0..20] * 0.05). */
int lyaf_flux_pdf(int64_t n_pix, const float *F, int64_t *counts, void *stream);

/* 1D line-of-sight flux power spectrum (Section 4.3; the paper prints no
 * estimator, the standard one is used): per skewer of N pixels of width dv,
 * delta_j = F_j / mean_F - 1 and
 *   P(k_m) = (dv / N) |sum_j delta_j exp(-2 pi i m j / N)|^2,
 *   k_m = 2 pi m / (N dv) (s/km),  m = 0 .. N/2,
 * computed in FP64 (an FFT per skewer) and stored as float.
 *   offsets: HOST [S+1] int64; every N must be a power of two in [2, 8192].
 *   dv:      DEVICE [S] float (> 0).
 *   F:       DEVICE [P] float.
 *   mean_F:  the mean flux that defines delta (> 0; e.g. the rescale target).
 *   power:   DEVICE float, written: skewer s holds N_s/2 + 1 values from
 *            sum_{s' < s} (N_s'/2 + 1).
 * Errors: EINVAL (host); LYAF_STATUS_DOMAIN when dv <= 0 or not finite. */
int lyaf_flux_power(int64_t n_skewers, const int64_t *offsets, const float *dv, const float *F,
                    double mean_F, float *power, void *stream);

/* ---- skewer-only field synthesis (Section 2.1, eqs. 1 and 3; Appendix B) ----
 *
 * The linear fields that feed the optical depths, generated in Fourier space
 * and brought back to real space only along the sight-lines that are needed.
 * A Gaussian field g(k) is given on the half-spectrum of a real n^3 grid of a
 * periodic box of side L, k = (2 pi / L)(mx, my, mz) with mx, my signed
 * (index i stands for i - n when i > n/2) and mz = 0 .. n/2:
 *
 *   delta_DM(k) = amp sqrt(P(|k|)) g(k),   P linearly interpolated from
 *                 pk[j] at |k| = j dk, 0 past the table's last node;
 *   delta_b(k)  = delta_DM(k) / (1 + k^2 / k_F^2)             (eq. 1)
 *   v_z(k)      = E_plus i (k_z / k^2) delta_DM(k), 0 at k = 0  (eq. 3, the
 *                 component along the sight-lines, which run along z);
 *
 * and on sight-line s, the column (sx[s], sy[s]), for z = 0 .. n-1,
 *
 *   f_s(z) = n^-3 sum_{mx, my} sum_{mz=0}^{n/2} c_mz Re[F(k) e^{2 pi i (mx x + my y + mz z)/n}]
 *
 * with c_mz = 1 at mz = 0 and n/2 and 2 otherwise (the real field whose
 * half-spectrum is F, numpy's irfftn).  The transforms run across the
 * (kx, ky) planes, keeping only the rows y that some sight-line uses, then
 * along each sight-line: FP32 data and arithmetic for the my transform, FP64
 * for the mx sums and the z transform, FP32 multipliers, float output.  The
 * table should reach the largest |k| of the grid, sqrt(3) pi n / L (or end
 * at zero power): a mode at the table's last node is decided in FP32. */
typedef struct {
  int64_t n;        /* grid points per side: a power of two, 4 .. 2048 */
  double box;       /* side L of the periodic box (> 0, finite) */
  double amp;       /* normalisation of delta_DM (finite) */
  double k_F;       /* filtering wavenumber of eq. (1) (> 0; +INFINITY: no filter) */
  double E_plus;    /* velocity factor of eq. (3) (finite) */
  double dk;        /* spacing of the power table (> 0, finite) */
  int64_t n_table;  /* entries of the power table (1 .. 2^31 - 1) */
} lyaf_field_params;

/* delta_b and v_z on n_lines sight-lines.
 *   modes: DEVICE complex float [n][n][n/2+1] (interleaved re, im; mz fastest),
 *          the half-spectrum g(k), read only.
 *   pk:    DEVICE double [n_table], the power table.
 *   sx, sy: HOST int32 [n_lines], columns in 0 .. n-1 (repeats allowed).
 *   delta_b, v_z: DEVICE float [n_lines][n], written (sight-line s at s*n).
 * The library keeps a workspace of 16 R n (n/2+1) + 32 n_lines (n/2+1) bytes,
 * R the number of distinct sy values (about 8.6 GB at n = 1024 with every
 * row in use).  Errors: EINVAL (host checks above), EDEVICE, ENOMEM. */
int lyaf_field_skewers(const lyaf_field_params *fp, const void *modes, const double *pk,
                       int64_t n_lines, const int32_t *sx, const int32_t *sy, float *delta_b,
                       float *v_z, void *stream);

/* ---- 3D flux power spectrum from sight-lines (Section 6.2, eq. 7) ----
 *
 * A mock survey's S sight-lines of n pixels run along z through the columns
 * (sx[s], sy[s]) of an n^3 periodic grid of side L.  The flux contrast
 * delta_s(z) = F_s(z) / mean_F - 1 of each sits in its column with weight w_s
 * (1 in the paper); the rest of the box is empty.  With unnormalised DFTs
 *   G_s(mz)   = sum_z delta_s(z) e^{-2 pi i mz z / n},
 *   W(mx, my) = sum_s w_s e^{-2 pi i (mx sx_s + my sy_s) / n},
 *   D(m)      = sum_s w_s G_s(mz) e^{-2 pi i (mx sx_s + my sy_s) / n},
 * the reconstruction of eq. (7) is
 *   P_true(m) = P_box(m) - [P_1D(mz) + p_noise] P_2D,w(mx, my),
 *   P_box = L^3 n^-6 |D|^2,  P_1D = L n^-2 mean_s |G_s|^2,  P_2D,w = L^2 n^-4 |W|^2
 * (the subtracted term equals P_box when every sight-line carries the same
 * spectrum: the aliasing it removes).  The modes of the half-spectrum
 * (mz = 0 .. n/2, weight 2 for 0 < mz < n/2, which stand for their conjugate
 * partners) are averaged in spherical shells of the fundamental wavenumber:
 * shell b holds b <= |m| < b + 1, |m| = sqrt(mx^2 + my^2 + mz^2), k = 2 pi m / L.
 * FP64 throughout; the shell sums are FP64 atomics, so repeated calls agree to
 * rounding, not bitwise. */
typedef struct {
  int64_t n;        /* pixels per sight-line = grid side: a power of two, 4 .. 2048 */
  double box;       /* side L (> 0, finite) */
  double mean_F;    /* mean flux defining the contrast (> 0, finite) */
  double p_noise;   /* flat 1D noise power P_N (>= 0, finite; 0 for noiseless flux) */
  int64_t n_bins;   /* shells (>= 1); shells past sqrt(3) n / 2 are empty */
} lyaf_power3d_params;

/*   F:       DEVICE float [n_lines][n], sight-line s at s*n.
 *   sx, sy:  HOST int32 [n_lines], columns in 0 .. n-1 (repeats add up).
 *   weights: DEVICE double [n_lines], or NULL for unit weights.
 *   counts, k_mean, p_true, p_box: DEVICE double [n_bins], written: each
 *     shell's mode count, mean |k|, mean P_true and mean P_box (0 for empty
 *     shells).
 * The library keeps a workspace of 16 (n_lines + n R)(n/2+1) + 8 n^2 bytes and
 * a few MB of shell partials, R the number of distinct sy values (about 8.7 GB
 * at n = 1024 with every row in use).  Errors: EINVAL (host checks above;
 * n_lines >= 1), EDEVICE, ENOMEM. */
int lyaf_flux_power_3d(const lyaf_power3d_params *pp, int64_t n_lines, const float *F,
                       const int32_t *sx, const int32_t *sy, const double *weights,
                       double *counts, double *k_mean, double *p_true, double *p_box,
                       void *stream);

/* ---- plans: the whole forward, tuned and captured once, replayed many times ----
 *
 * Section 2.3 applies the same steps to every spectrum of a survey: eq. (6) per
 * skewer, then one mean-flux rescale over all of them.  A plan binds one batch
 * of skewers (their device arrays and host offsets), the parameters, the
 * target mean flux and the output buffers, and records the whole forward
 * (reach pass, windowed tau kernel, mean-flux root-find, tau' and F) as one
 * hipGraph.  lyaf_plan_execute replays it: the array contents may change
 * between executions, their addresses and the offsets may not.
 *
 * The windowed tau kernel runs as one persistent launch: a grid sized to the
 * resident workgroups takes (skewer, tile) items from a device queue ordered by
 * estimated cost (largest first), so ragged batches finish evenly.  With
 * LYAF_PLAN_AUTOTUNE the kernel shape (source streams, targets per lane, tile
 * length) and the launch form (persistent or one workgroup per item) are timed
 * on the plan's own data at creation and the winner is cached in a text file
 * ($LYAF_TUNE_CACHE, else $HOME/.cache/lyaf_tune.txt) under a key made of the
 * device name, compute-unit count, batch shape buckets and window; later plans
 * with the same key reuse it without timing.  Without the flag the default
 * shape with the persistent launch is used.
 *
 * All plan memory is allocated in lyaf_plan_create; execution allocates
 * nothing.  Creation runs kernels on `stream` (and synchronises it); the
 * outputs then hold a valid result. */
typedef struct lyaf_plan lyaf_plan;

#define LYAF_PLAN_AUTOTUNE 1u  /* time the kernel shapes at creation (cached) */
#define LYAF_PLAN_NO_GRAPH 2u  /* execute by re-enqueueing the kernels, no hipGraph */

/* tau_out, F_out: DEVICE [P] float; A_dev: DEVICE double.  target_F in (0, 1).
 * Errors: as lyaf_tau and lyaf_normalise_mean_flux, plus EDEVICE/ENOMEM from
 * graph capture or allocation. */
int lyaf_plan_create(const lyaf_skewers *sk, const lyaf_params *prm, double target_F,
                     float *tau_out, float *F_out, double *A_dev, uint32_t plan_flags,
                     void *stream, lyaf_plan **plan_out);
/* Replay the forward on `stream` (any stream of the plan's device). */
int lyaf_plan_execute(lyaf_plan *plan, void *stream);
/* Read and clear the plan's status word (LYAF_STATUS_*); synchronises `stream`. */
int lyaf_plan_status(lyaf_plan *plan, void *stream, uint32_t *device_status);
/* NUL-terminated one-line description of the chosen configuration (JSON);
 * returns the length it needs (excluding the NUL) or a negative code. */
int lyaf_plan_describe(const lyaf_plan *plan, char *buf, int64_t buf_len);
/* Free the plan (synchronises the device first).  NULL is accepted. */
int lyaf_plan_destroy(lyaf_plan *plan);

/* Read and clear the device status word of the current device's workspace
 * for `stream`.  Synchronises `stream`.  *device_status receives LYAF_STATUS_*
 * bits accumulated since the last read. */
int lyaf_status_read(void *stream, uint32_t *device_status);

/* ---- kernel timing (measurement support) ----
 *
 * lyaf_kernel_timing(1) clears earlier records and starts recording: each
 * launch site of the entry points then records a pair of HIP events on the
 * caller's stream around its kernels, under one of the names
 *   "reach"      the per-skewer constants and reach pass (lyaf_tau, lyaf_tau_backward)
 *   "tau"        the windowed tau kernel of lyaf_tau (one-launch grid form: the
 *                events are set by the runtime at the kernel's own start and end,
 *                hipExtLaunchKernel; persistent form: around the queue reset and
 *                the kernel); "tau_plain" the plain full-sum kernels
 *   "normalise", "normalise_backward", "tau_adjoint", "instrument",
 *   "instrument_backward", "flux_pdf", "flux_power",
 *   "field_ky", "field_kx", "field_z" (the three kernels of lyaf_field_skewers),
 *   "flux_power_3d" (every kernel of lyaf_flux_power_3d).
 * Launches under stream capture (plans, caller graphs) are not recorded, and
 * recording stops after 65536 launches.  lyaf_kernel_timing(0) stops and
 * clears.  lyaf_kernel_timing_read waits for the recorded launches of `name`,
 * writes the sum of their durations (ms) and their number, and drops those
 * records.  Timing costs two event records per launch; it is off by default.
 * Errors: EINVAL (NULL argument), EDEVICE. */
int lyaf_kernel_timing(int enable);
int lyaf_kernel_timing_read(const char *name, double *total_ms, int64_t *count);

/* Human-readable name of a return code (static string). */
const char *lyaf_strerror(int code);

/* Library version, as MAJOR*10000 + MINOR*100 + PATCH. */
int lyaf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LYAF_H */
