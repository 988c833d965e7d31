// lyaf_internal.h -- declarations shared by the HIP translation units of liblyaf.
//
// Physical constants, per-skewer constants, workspace layout and the host-side
// launchers that lyaf_api.hip calls.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lyaf.h"

namespace lyaf {

// ---------------------------------------------------------------------------
// Constants.  beta = sqrt(2 k_B / m_H) in km s^-1 K^-1/2, with
// k_B = 1.380649e-16 erg/K (CODATA 2018, exact) and m_H = 1.6735575e-24 g
// (hydrogen atom), so that b = beta sqrt(T) is the thermal Doppler parameter of
// Section 2.3 (b = 12.845 km/s at 1e4 K).
constexpr double kBeta = 0.12845065404917816;
constexpr double kSqrtLog2e = 1.2011224087864498;  // sqrt(1 / ln 2)
constexpr double kSqrtPi = 1.7724538509055159;
constexpr double kLn2 = 0.69314718055994531;
constexpr double kLog2e = 1.4426950408889634;

// Exponents of eq. (4): n_HI ~ Delta^2 T^-0.7, divided by b ~ T^0.5.
constexpr float kTempExpW = -1.2f;  // d ln w / d ln T
constexpr float kTempExpR = -0.5f;  // d ln (1/b) / d ln T

// Tiling of the windowed optical-depth kernel.
constexpr int kWave = 64;
constexpr int kTauThreads = 256;   // 4 waves per workgroup
constexpr int kTauTile = 512;      // targets per workgroup (one work item)
constexpr int kGroup = 8;          // sources per window-bounds group (= source streams)
constexpr int kChunk = 1536;       // sources staged in LDS at once

// Per-skewer constants, computed in FP64 by the reach kernel and rounded once.
struct SkewerConst {
  float W;       // tau_ref 1e4^0.7 dv / (sqrt(pi) beta) T0^-1.2 : w = W Delta^2 D^(-1.2(gamma-1))
  float R;       // sqrt(log2 e) / (beta sqrt(T0))              : r = R D^(-0.5(gamma-1))
  float B;       // beta sqrt(T0)                               : b = B D^(0.5(gamma-1))
  float gm1;     // gamma - 1
  float dv;      // pixel width (km/s)
  float inv_dv;  // 1 / dv
  int32_t reach; // max_j (|v_j| + k b_j) / dv, rounded up, plus margin (pixels)
  int32_t n;     // pixels in the skewer
};

// Mean-flux root-find state (device).  The iteration runs on a sample of the
// pixels, then with FP32 moments over all pixels, then FP64 moments.
struct NormState {
  double A, lo, hi;  // iterate and bracket
  double P, Ps;      // pixels in the batch and in the sample
  double target;
  double step;       // |A_new - A_old| / A_new of the last step
  int32_t iter, done, status;
  int32_t phase;     // kNormPhaseFP32, kNormPhaseExact
  int32_t pending;   // no moments at A yet (the next full pass computes them)
  int32_t buf;       // partial buffer (0 or 1) holding the last moments
  int32_t nparts;    // workgroups that wrote them
};
constexpr int32_t kNormPhaseFP32 = 1, kNormPhaseExact = 2;

// Per-(device, stream) workspace.
struct Workspace {
  int device = -1;
  hipStream_t stream = nullptr;
  uint32_t *status = nullptr;       // sticky LYAF_STATUS_* bits
  double *partials = nullptr;       // [kPartialsDoubles]
  NormState *norm = nullptr;        // [kNormPasses + 2]
  double *ratio = nullptr;          // backward-normalise scalar
  // growable buffers (the work lists of the entry points live in the API's
  // per-(workspace, tile) records; a plan keeps its offsets here)
  SkewerConst *skc = nullptr;  int64_t skc_cap = 0;
  int64_t *offsets = nullptr;  int64_t off_cap = 0;
  double *gpart = nullptr;     int64_t gpart_cap = 0;  // adjoint per-item FP64 partials
  unsigned int *queue = nullptr;                      // persistent work-queue counter
  // flux statistics: PDF partial counts, power-spectrum offsets (host mirror in the API)
  uint32_t *pdf_part = nullptr; int64_t pdf_part_cap = 0;
  int64_t *ps_off = nullptr;   int64_t ps_off_cap = 0;
  int64_t *ps_mo = nullptr;    int64_t ps_mo_cap = 0;
  double2 *ps_twiddle = nullptr;                      // [kPsMaxN / 4], built once
  // field synthesis: the intermediates of both fields (my-transformed rows,
  // then the mx-transformed sight-lines)
  float2 *field_T = nullptr;   int64_t field_T_cap = 0;
  double2 *field_C = nullptr;  int64_t field_C_cap = 0;
  // 3D flux power: complex (G, D1) and real (P1d, P2d, shell partials) buffers
  double2 *p3d_c = nullptr;    int64_t p3d_c_cap = 0;
  double *p3d_r = nullptr;     int64_t p3d_r_cap = 0;
  double *p3d_geom = nullptr;  int64_t p3d_geom_cap = 0;  // shells' counts and |m| sums
  int p3d_geom_n = 0, p3d_geom_nb = 0;                    // grid they belong to (0: none)
};
constexpr int kMaxPartialBlocks = 512;  // workgroups of a root-find pass
constexpr int kPartStride = 8;          // doubles per workgroup partial
constexpr int kNormPasses = 3;          // full root-find passes after the sample
constexpr int kSampleN = 8192;          // pixels the root-find samples first
constexpr int kSampleCap = 16384;       // room for the sample in the partials allocation
// The partials allocation also holds the sample (up to kSampleCap floats)
// after the two partial buffers.
constexpr int64_t kPartialsDoubles = 2 * kPartStride * kMaxPartialBlocks + kSampleCap / 2;
static_assert(kSampleN <= kSampleCap, "the sample fits its room");
constexpr double kNormAcceptStep = 1e-5;
// Largest batch of the mean-flux root-find: the sample index k P / kSampleN is
// formed in int64 (2^48 pixels is a petabyte of tau, far beyond any device).
constexpr int64_t kMaxNormPixels = int64_t(1) << 48;

// Kernel-side view of a skewer batch.
struct Batch {
  const float *delta, *vpec, *dv, *T0, *gamma;
  const int64_t *offsets;  // device [S+1]
  SkewerConst *skc;        // device [S]
  int64_t n_skewers;
  float tau_ref, pivot, window_k;
  uint32_t *status;
};

// ---------------------------------------------------------------------------
// Launchers (return hipError_t of the launch).
hipError_t launch_reach(const Batch &b, hipStream_t st);
// Shapes of the windowed kernel that the tuner chooses from: S source streams
// per wave, M targets per lane, TILE targets per work item.
struct TauVariant {
  int S, M, tile;
};
constexpr int kNumTauVariants = 6;
constexpr int kTauVariantDefault = 4;  // shape used when no shape is forced or tuned
extern const TauVariant kTauVariants[kNumTauVariants];

// persistent_grid > 0 launches the persistent work-queue form with that many
// workgroups (queue: a device counter, reset by a kernel inside the launch).
// start / stop (grid form only, not under stream capture): events that the
// runtime sets at the kernel's own start and end (hipExtLaunchKernel).
hipError_t launch_tau_window(const Batch &b, const int2 *items, int64_t n_items,
                             float *tau, hipStream_t st, int variant = kTauVariantDefault,
                             int persistent_grid = 0, unsigned int *queue = nullptr,
                             hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Resident workgroups of the persistent form on the current device.
int tau_persistent_grid(int variant);
hipError_t launch_tau_plain(const Batch &b, int64_t skewer, int64_t n, float *tau,
                            hipStream_t st);
hipError_t launch_norm(int64_t n_pix, float *tau, float *F, double target_F,
                       double *A_dev, Workspace &ws, hipStream_t st);
// lyaf_normalise_mean_flux_noalloc: the same kernels with their scratch in a
// static device array of kNormNoAllocScratchBytes per device (no allocation);
// status may be null (the bits then land in the array and are not reported).
constexpr size_t kNormNoAllocScratchBytes = LYAF_NORM_NOALLOC_SCRATCH_BYTES;
hipError_t launch_norm_noalloc(int64_t n_pix, float *tau, float *F, double target_F,
                               double *A_dev, uint32_t *status, hipStream_t st);
hipError_t launch_norm_backward(int64_t n_pix, const float *tau, const double *A_dev,
                                const float *gF, const float *gT, int implicit_A,
                                float *out, Workspace &ws, hipStream_t st);
// Instrument model (Gaussian line-spread convolution, resampling, noise).
constexpr int kInsMaxRatio = 252;                         // largest bin width in pixels
constexpr double kInvTwoSqrtLn2 = 0.60056120439322491;    // b_L = FWHM / (2 sqrt(ln 2))
constexpr double kSpeedOfLightKms = 299792.458;
constexpr double kLymanAlphaAngstrom = 1215.67;  // rest wavelengths (vacuum)
constexpr double kLymanBetaAngstrom = 1025.72;
struct InsArgs {
  const int64_t *offsets;      // device [S+1] pixel offsets
  const int64_t *out_offsets;  // device [S+1] bin offsets
  const float *dv;             // device [S]
  const float *in;             // forward: F [P]; backward: grad of the bins [P_out]
  float *out;                  // forward: bins [P_out]; backward: grad of F [P]
  const float *noise;          // forward: [P_out] or null
  double fwhm, bin, inv_bin, v_start, sigma, window_k;
  uint32_t *status;
};
int ins_items_per_skewer(int64_t n, int64_t n_out, bool backward);
// Whether the backward's per-skewer kernel takes a skewer (its bins fit that
// kernel's LDS); the per-tile kernel's items cover the others.
bool ins_bwd_skewer_item(int64_t n, int64_t n_out);
// skewer_items: the backward's per-skewer items, max_bins the most bins of
// their skewers (ignored by the forward).
hipError_t launch_instrument(const InsArgs &a, const int2 *items, int64_t n_items,
                             const int2 *skewer_items, int64_t n_skewer_items, int max_bins,
                             bool backward, hipStream_t st);
// Flux statistics (flux PDF, 1D flux power spectrum).
constexpr int kPdfMaxBlocks = 1024;  // workgroups of the PDF counting kernel
constexpr int kPdfCountSlots = 24;   // 21 bins, below, above, NaN
constexpr int kPsMaxN = 8192;        // longest skewer of the power spectrum
hipError_t launch_flux_pdf(int64_t n, const float *F, uint32_t *part, int64_t *counts,
                           hipStream_t st);
hipError_t launch_twiddles(double2 *T, hipStream_t st);  // kPsMaxN / 4 entries
hipError_t launch_flux_power(int64_t n_skewers, int max_n, const float *F, const int64_t *offsets,
                             const int64_t *mode_off, const float *dv, double inv_mean,
                             const double2 *T, float *P, uint32_t *status, hipStream_t st);
// Skewer-only field synthesis (eqs. 1 and 3, Appendix B).
constexpr int kFieldMaxN = 2048;  // grid points per side
struct FieldArgs {
  const float2 *modes;   // device [N][N][N/2+1] Gaussian modes g(k)
  const double *pk;      // device [n_table] power table, P at |k| = j dk
  int N, H;              // grid side and N/2 + 1
  int n_table, n_rows;   // table entries; rows y that some sight-line uses
  float kfun;            // 2 pi / L
  float inv_dk;          // 1 / dk
  float amp;             // delta_DM = amp sqrt(P) g
  float kfun2_inv_kF2;   // (2 pi / L)^2 / k_F^2 (0: no filter)
  float E_over_kfun;     // E_+ / (2 pi / L)
  double inv_n3;         // N^-3
  const int *rows;       // device [n_rows]: y of each kept row
  const int4 *groups;    // device [n_groups]: (row index, first line, count, 0)
  const int2 *lines;     // device [S]: (sight-line, x), grouped by row
  float2 *Tb, *Tv;       // device [n_rows][N][H] after the my transform
  double2 *Cb, *Cv;      // device [S][H] after the mx transform
  float *delta_b, *v_z;  // device [S][N] outputs
  const double2 *twiddle;  // the shared FFT table (kFftTableLen / 2 entries)
};
int field_ky_columns(int N);  // mz values per field_ky work item
// Sets the kernels' LDS limits once per device; *ky_resident: resident
// workgroups of the persistent my-transform kernel.
hipError_t field_kernel_attributes(int *ky_resident);
hipError_t launch_field_ky(const FieldArgs &a, int resident, hipStream_t st);
hipError_t launch_field_kx(const FieldArgs &a, int n_groups, hipStream_t st);
hipError_t launch_field_z(const FieldArgs &a, int n_lines, hipStream_t st);
constexpr int kFieldLinesPerGroup = 8;
// 3D flux power spectrum of eq. (7) from sight-lines.
constexpr int kP3dMaxN = 2048;        // pixels per sight-line = grid side
constexpr int kP3dMaxLds = 160 * 1024;  // LDS of one workgroup
constexpr int kP3dP1dChunk = 256;       // sight-lines per partial sum of P_1D
struct P3dArgs {
  const float *F;         // device [S][n] flux
  const double *w;        // device [S] weights or null (all 1)
  int n, H;               // grid side and n/2 + 1
  int n_rows, n_lines, n_bins;
  double inv_mean;        // 1 / Fbar
  double L, p_noise;      // box side, flat 1D noise power
  const int *rows;        // device [n_rows]: y of each row in use
  const int *row_of_y;    // device [n]: row index of y, -1 for rows without sight-lines
  const int *row_first;   // device [n_rows + 1]: the row's sight-lines in `lines`
  const int2 *lines;      // device [S]: (sight-line, x), grouped by row
  double2 *G;             // device [S][H]: the sight-lines' transforms
  double *P1d;            // device [H]
  double *p1d_part;       // device [ceil(S / 256)][H] partial sums of P_1D
  double *P2d;            // device [n][n] (mx, my)
  double2 *D1;            // device [n][n_rows][H]: sum over a row's sight-lines
  double *shells;         // device [workgroups][2][shells]: P_true, P_box sums
  double *geom_part;      // device [workgroups][2][shells]: counts, |m| sums
  double *geom;           // device [2][shells], kept across calls
  double *counts, *k_mean, *p_true, *p_box;  // device [n_bins] outputs
  const double2 *twiddle;  // the shared FFT table
};
int p3d_shell_bins(int n, int n_bins);  // shells kept in LDS
int p3d_y_columns(int n);               // mz per item of the y transform
// Sets the kernels' LDS limits once per device; *y_grid: resident workgroups
// of the y-transform kernel for grid side n and nb shells.
hipError_t p3d_kernel_attributes(int n, int nb, int *y_grid);
// need_geom: (re)compute the shells' counts and |m| sums into a.geom first.
hipError_t launch_power3d(const P3dArgs &a, int y_grid, bool need_geom, hipStream_t st);
hipError_t launch_tau_adjoint(const Batch &b, const int2 *items, int64_t n_items,
                              const int64_t *item_base_dev, const float *g,
                              float *gdelta, float *gvpec, double *gT0,
                              double *ggamma, double *gpart, hipStream_t st);

}  // namespace lyaf
