/*
 * cemu_measure.h -- measurement entry point of libcemu, beside the gate API
 * of cemu.h: the peak rates that the blind-rotation kernels' fractions of
 * peak are quoted against, measured on the current device.
 */
#ifndef CEMU_MEASURE_H
#define CEMU_MEASURE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Peak-rate probes on the current HIP device, at the occupancy of the
 * throughput kernels (one workgroup of eight waves per compute unit):
 *   fp64_flops_per_s: host double, FP64 fused multiply-adds per second x 2,
 *     from sixteen independent chains per lane (65,536 iterations each);
 *   int8_ops_per_s: host double, int8 multiply-adds per second x 2 of
 *     v_mfma_i32_16x16x64_i8, eight independent accumulators per wave
 *     (16,384 iterations each).
 * Each probe is launched eight times, alternating, timed with hipEvents on
 * hip_stream (NULL = the default stream), and its fastest launch counts (the
 * first ones run while the clocks ramp up from idle). The call waits for
 * them (about 0.1 s) and allocates a small device buffer for their results.
 * Errors: CEMU_ERR_NULL, CEMU_ERR_OOM, CEMU_ERR_HIP. */
int cemu_measure_peaks(double *fp64_flops_per_s, double *int8_ops_per_s, void *hip_stream);

/* LDS bandwidth of the current HIP device, summed over its compute units, at
 * the same occupancy: every wave writes (write_bytes_per_s), or reads
 * (read_bytes_per_s), its own 8 KiB region of a 64 KiB LDS buffer as eight
 * rows of 64 consecutive 16-byte slots per iteration (no bank conflicts;
 * per-lane base plus immediate offsets, no address arithmetic between the
 * accesses), 4,096 iterations. Timing, repetitions and errors as
 * cemu_measure_peaks. The FFT kernels' LDS traffic is quoted against these. */
int cemu_measure_lds(double *write_bytes_per_s, double *read_bytes_per_s, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* CEMU_MEASURE_H */
