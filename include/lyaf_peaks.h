/* lyaf_peaks.h -- measured device rates that bound the optical-depth kernels.
 *
 * A measurement library (libpeaks.so), separate from liblyaf.so: the
 * benchmark states its pair-rate roofline from these rates, measured on the
 * device it runs on, next to the vendor's published peaks.
 *
 *   c_valu = 1 / (rate of independent FP32 FMAs, lane operations per second)
 *   trans  = rate of independent exp2 (the transcendental unit alone)
 *   mix    = exp2 rate when each exp2 is issued beside N independent FMAs:
 *            if the transcendental unit overlaps the other VALU work this
 *            stays at the trans rate until N c_valu exceeds 1 / trans
 *   c_exp  = extra time per lane of one exp2 in the pair arithmetic of the
 *            tau sum (t = k a + t0; e = exp2(-t t); acc += w e), measured as the
 *            difference between that loop with and without the exp2
 *   pair_peak = min(fma rate / 3, trans rate): the pair rate of the direct
 *            form (each pair its own exp2 and at least three other VALU
 *            operations: t_k, its square and the accumulate) when the two
 *            units overlap; a ceiling for that form, since it counts no
 *            staging, compensation or addressing
 *
 * All rates are for the whole device.  Packed FP32 instructions are not used.
 */
#ifndef LYAF_PEAKS_H
#define LYAF_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LYAF_PEAKS_MIX_N 6 /* exp2 beside N = 0, 1, 2, 3, 4, 6 FMAs */

typedef struct lyaf_peak_rates {
  double fma_lane_ops_per_s;   /* v_fma_f32, 8 independent chains per lane */
  double pair_per_s_exp;       /* pair loop with the exp2, lane-pairs per second */
  double pair_per_s_noexp;     /* the same loop with the exp2 replaced by its argument */
  double c_valu_s;             /* seconds per lane operation: 1 / fma_lane_ops_per_s */
  double c_exp_s;              /* seconds per lane exp2 inside the pair loop */
  double pair_peak_per_s;      /* min(fma_lane_ops_per_s / 3, trans_lane_ops_per_s) */
  double trans_lane_ops_per_s; /* v_exp_f32, 4 independent chains per lane */
  double mix_fma_per_exp[LYAF_PEAKS_MIX_N]; /* N: FMAs issued per exp2 */
  double mix_exp_per_s[LYAF_PEAKS_MIX_N];   /* exp2 per second beside N FMAs each */
  double copy_bytes_per_s;     /* streaming copy, bytes read + written per second */
  int32_t compute_units;       /* of the device measured */
  int32_t clock_khz;           /* its peak engine clock */
} lyaf_peak_rates;

/* Runs the microbenchmarks on the current device and `stream` (hipStream_t,
 * NULL = default stream); synchronises the stream; allocates and frees 1 GiB of
 * device memory for the copy.  Returns 0, -1 if out is NULL, -5 on a device
 * error, -6 if the buffers cannot be allocated. */
int lyaf_peaks_measure(lyaf_peak_rates *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
