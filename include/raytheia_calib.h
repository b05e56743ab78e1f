/*
 * raytheia_calib.h -- measurement probes of the MI355X reverse ray-walk
 * library.
 *
 * These calls compute nothing of the method.  They measure the two
 * ceilings against which the walk kernels are placed: the HBM bandwidth a
 * plain stream achieves, and the rate at which the chip issues vector (VALU)
 * instructions.  The benchmark runs them beside the walks, on the same GPU
 * and in the same process.  Conventions as in raytheia.h: rt_status codes,
 * rt_last_error, device pointers borrowed from the caller, work queued on
 * the given stream (a hipStream_t passed as void*, NULL = default stream).
 */
#ifndef RAYTHEIA_CALIB_H
#define RAYTHEIA_CALIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes that one block of the stream probes moves (16 KB): the buffers of
 * rt_calib_copy and rt_calib_read are a whole number of these. */
size_t rt_calib_stream_granule(void);

/* Copies bytes from d_src to d_dst (device, 16-byte aligned, not
 * overlapping) with 16-byte non-temporal loads and stores, four per lane in
 * flight: bytes read + bytes written over the kernel's duration is the
 * achievable copy bandwidth.  bytes: a positive multiple of the granule,
 * at most 2^31 - 1 granules.  Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_calib_copy(const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Reads bytes from d_src (device, 16-byte aligned) with the loads of
 * rt_calib_copy and writes the XOR of each block's words to
 * d_sink[bytes / granule] (device uint32): the achievable read bandwidth.
 * Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_calib_read(const void *d_src, size_t bytes, uint32_t *d_sink, void *stream);

/* VALU issue probe: n_threads lanes (a positive multiple of 256, at most
 * 2^31 - 256; blocks of 256) each run iters iterations of 8 independent
 * dependency chains of one instruction type and write one word to
 * d_out[n_threads] (device uint32):
 *   kind 0: v_fma_f64, 8 per wavefront and iteration;
 *   kind 1: v_xad_u32 ((a ^ k) + b), 8 per wavefront and iteration, plus
 *           one v_mov_b32 (a rotation of the chains);
 *   kind 2: v_fma_f32 (one lane op each; packed FP32 is disabled), 8 per
 *           wavefront and iteration.
 * The loop counter is scalar, so with enough wavefronts per SIMD to hide
 * the chains' latency the wavefront-instructions issued per second (the
 * count above over the kernel's duration) is the chip's VALU issue rate for
 * that instruction.  Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_calib_valu(int kind, int64_t n_threads, int iters, uint32_t *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAYTHEIA_CALIB_H */
