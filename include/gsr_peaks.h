/*
 * gsr_peaks.h -- achievable-peak probes of the GPU (part of libgsr.so).
 *
 * Measurement only: these calls are not on the rendering path. They give the
 * denominators of the roofline fractions the benchmark reports, measured on
 * the device in use instead of read off the data sheet. Each probe allocates
 * its own buffers (hipMalloc, freed before it returns), runs its kernel once
 * to warm up and then `reps` times between two HIP events on `stream` (a
 * hipStream_t, 0 = legacy default stream), synchronises, and writes the
 * average rate. Return value: 0, or a negative code below.
 */
#ifndef GSR_PEAKS_H
#define GSR_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GSR_PEAKS_ERR_INVALID = -1,   /* bad argument */
  GSR_PEAKS_ERR_OOM = -2,       /* device allocation failed */
  GSR_PEAKS_ERR_HIP = -3        /* a HIP runtime call failed */
};

/* HBM bandwidth of a device-to-device copy of `bytes` (1 MiB .. 64 GiB) with
 * 16-byte loads and stores: *bytes_per_s = bytes read + bytes written per
 * second. */
int gsr_peak_copy(int64_t bytes, int32_t reps, void* stream, double* bytes_per_s);

/* FP32 VALU issue rate: eight independent fused multiply-add chains per lane,
 * one non-packed instruction per lane and step, eight waves per SIMD on every
 * CU. *lane_ops_per_s = lane instructions per second (each an FMA, 2 FLOPs). */
int gsr_peak_valu(int32_t reps, void* stream, double* lane_ops_per_s);

/* Rate of the hardware 2^x (the exponential of the blend kernels), measured
 * like gsr_peak_valu: *lane_ops_per_s = 2^x lane operations per second. */
int gsr_peak_exp(int32_t reps, void* stream, double* lane_ops_per_s);

/* LDS read bandwidth: bank-conflict-free 16-byte reads by every lane, two
 * 256-thread workgroups of 64 KiB each per CU (x4 rounds of CUs).
 * *bytes_per_s = LDS bytes read per second over the whole device. */
int gsr_peak_lds(int32_t reps, void* stream, double* bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* GSR_PEAKS_H */
