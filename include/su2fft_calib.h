/*
 * su2fft calibration kernels (exported by the same library as su2fft.h).
 *
 * Not part of the transform.  They measure what the device sustains, so that
 * the transform's kernels can be priced against achievable as well as
 * published peaks: a streaming copy and a streaming fill for HBM, and
 * back-to-back matrix-core products for the three precisions the
 * beta-contraction kernels use.
 *
 * Same conventions as su2fft.h: plain pointers and sizes, the HIP stream
 * (hipStream_t; NULL = the null stream), asynchronous launches, arguments
 * validated before any HIP call, SU2_ERR_HIP with su2_last_hip_error() set
 * when a launch fails.  The caller owns every buffer.
 */
#ifndef SU2FFT_CALIB_H
#define SU2FFT_CALIB_H

#include <stdint.h>

#include "su2fft.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` from d_src to d_dst (device memory, 16-byte aligned, `bytes`
 * a positive multiple of 16, the two ranges disjoint) with non-temporal
 * 16-byte loads and stores.  Moves 2 x bytes through HBM.
 * SU2_ERR_INVALID_VALUE on a null or misaligned pointer, a bad size or
 * overlapping ranges. */
su2_status_t su2_calib_copy(const void* d_src, void* d_dst, int64_t bytes, hipStream_t stream);

/* Write `value` to every float of d_dst (device memory, 16-byte aligned,
 * `bytes` a positive multiple of 16) with non-temporal 16-byte stores. */
su2_status_t su2_calib_fill(void* d_dst, int64_t bytes, float value, hipStream_t stream);

/* Matrix-core throughput.  kind 0 = FP64 16x16x4, 1 = FP32 16x16x4,
 * 2 = BF16 16x16x32 with FP32 accumulation.  `workgroups` workgroups of 256
 * threads each run `iters` iterations of 4 independent products per wave;
 * lane l of every wave feeds a = l mod 3 + 1 and b = l mod 5 + 1 to every
 * operand element.  Each thread writes the sum of its accumulator elements to
 * d_out[thread] (workgroups x 256 floats, device memory, 16-byte aligned).
 * If `flops` (host) is not NULL it receives the flops the launch executes:
 * workgroups x 4 waves x iters x 4 x 2 x 16 x 16 x K.
 * SU2_ERR_INVALID_VALUE unless 0 <= kind <= 2, 1 <= workgroups <= 2^20,
 * 1 <= iters <= 2^24 and d_out is a non-null aligned pointer. */
su2_status_t su2_calib_mfma(int32_t kind, int32_t workgroups, int32_t iters, float* d_out, double* flops,
                            hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SU2FFT_CALIB_H */
