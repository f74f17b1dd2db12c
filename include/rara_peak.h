/*
 * rara_peak.h -- attainable-peak probes of the MI355X (gfx950), used to state
 * the renderer's roofline fractions against measured ceilings beside the
 * published ones.  Not part of the rendering path (include/rara.h); built as
 * a library of its own, libpeak.so.
 *
 * Both calls only enqueue one kernel on `stream` (a hipStream_t, NULL = the
 * default stream) and return 0, 1 for a bad argument, or 3 when the launch
 * failed.  The caller times them (HIP events on the same stream).
 */
#ifndef RARA_PEAK_H
#define RARA_PEAK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming copy of `bytes` (a multiple of 16) from device buffer src to
 * device buffer dst, 16-byte loads and stores, `blocks` workgroups of 256
 * threads striding over the buffer.  HBM bytes moved: 2 * bytes. */
int rara_peak_copy(void* dst, const void* src, size_t bytes, int blocks, void* stream);

/* `blocks` workgroups of 256 threads, each lane running 16 independent
 * chains of `iters` unpacked FP32 fused multiply-adds (no memory traffic;
 * `out`, a device buffer of blocks * 256 floats, is never written for the
 * arguments used).  Flops: rara_peak_fma_flops(blocks, iters), FMA = 2. */
int rara_peak_fma(float* out, int blocks, int iters, void* stream);
double rara_peak_fma_flops(int blocks, int iters);

#ifdef __cplusplus
}
#endif

#endif /* RARA_PEAK_H */
