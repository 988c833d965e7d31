/* lyaf_peaks.h -- measured device rates that bound the optical-depth kernels.
 *
 * A measurement library (libpeaks.so), separate from liblyaf.so: the
 * benchmark states its pair-rate roofline from these rates, measured on the
 * device it runs on, next to the vendor's published peaks.
 *
 *   c_valu = 1 / (rate of independent FP32 FMAs, lane operations per second)
 *   c_exp  = extra time per lane of one exp2 in the pair arithmetic of the
 *            tau sum (t = k a + t0; e = exp2(-t t); acc += w e), measured as the
 *            difference between that loop with and without the exp2
 *   pair_peak = 1 / (c_exp + 4 c_valu): pairs per second if every pair cost
 *            one exp2 and four FP32 operations and nothing else
 *
 * All rates are for the whole device.  Packed FP32 instructions are not used.
 */
#ifndef LYAF_PEAKS_H
#define LYAF_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lyaf_peak_rates {
  double fma_lane_ops_per_s;   /* v_fma_f32, 8 independent chains per lane */
  double pair_per_s_exp;       /* pair loop with the exp2, lane-pairs per second */
  double pair_per_s_noexp;     /* the same loop with the exp2 replaced by its argument */
  double c_valu_s;             /* seconds per lane operation: 1 / fma_lane_ops_per_s */
  double c_exp_s;              /* seconds per lane exp2 inside the pair loop */
  double pair_peak_per_s;      /* 1 / (c_exp + 4 c_valu) */
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
