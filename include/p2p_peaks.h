/*
 * p2p_peaks.h -- microbenchmarks of libp2p_peaks (gfx950): the measured
 * denominators quoted beside the published MI355X peaks in the rooflines of
 * libp2p's kernels.  Not part of the operator; nothing in libp2p uses them.
 *
 * Each entry point launches `blocks` workgroups of 256 threads on `stream`
 * (a hipStream_t, NULL = the null stream) and returns at once; the caller
 * times the launch with events.  `out` is a DEVICE buffer owned by the
 * caller, of at least blocks * 256 floats: every thread writes one value
 * there so that the compiler keeps the loop.  Return value: 0, or the
 * hipError_t of the launch; blocks < 1, iters < 1 or out == NULL return -1
 * without launching.
 */
#ifndef P2P_PEAKS_H
#define P2P_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* FP32 VALU issue: per thread, iters x 128 fused multiply-adds (v_fma_f32)
 * in 8 independent chains.  One FMA is one lane-slot. */
int p2pk_valu_fma(float *out, int64_t blocks, int32_t iters, void *stream);

/* FP32 reciprocal square root (v_rsq_f32): per thread, iters x 64 in 8
 * independent chains.  Its rate against p2pk_valu_fma gives the lane-slots
 * one rsq costs. */
int p2pk_valu_rsq(float *out, int64_t blocks, int32_t iters, void *stream);

/* FP32 matrix cores: per wavefront, iters x 32 v_mfma_f32_16x16x4f32 in 4
 * independent accumulators (2048 flop each). */
int p2pk_mfma_f32(float *out, int64_t blocks, int32_t iters, void *stream);

#ifdef __cplusplus
}
#endif

#endif
