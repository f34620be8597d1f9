/*
 * pf_probe.h -- measurement probes of libpencilfilter.so.
 *
 * Plain kernels that measure what this device sustains for the instruction
 * and access mixes the filters use: the ALU rate of one instruction issued
 * back to back on independent registers, and a flat HBM copy. They compute
 * nothing of the method; a benchmark times them (events on `stream`) to
 * read a filter's timing against an achieved rate as well as a published
 * peak. Conventions (status codes, thread-local message) are those of
 * pf.h. Launches are asynchronous on `stream` (NULL: the null stream).
 */
#ifndef PENCILFILTER_PF_PROBE_H
#define PENCILFILTER_PF_PROBE_H

#include "pf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PF_PROBE_DOT4 0  /* v_dot4 int8 (4 multiply-adds into an int32), as the uint8 filter */
#define PF_PROBE_FMA 1   /* v_fma_f32, as the FP32 filters                                 */

/* One launch of `blocks` workgroups of 256 lanes; each lane issues
 * iters x 128 instructions of kind `op` on 8 independent accumulators, so
 * one launch is blocks x 256 x iters x 128 lane-instructions. `out` is a
 * device buffer of blocks x 256 4-byte values that receives the lanes'
 * results (kept so that the work is not removed). blocks and iters in
 * 1..2^20; PF_EINVAL otherwise. */
pf_status pf_probe_alu(int32_t op, int32_t blocks, int32_t iters, void *out, void *stream);

/* out[i] = in[i] for i < n: device pointers, 16-byte aligned, not
 * overlapping; 16-byte non-temporal loads and stores, 4 per lane in flight.
 * Moves 8 n bytes (n reads, n writes of 4 bytes). */
pf_status pf_probe_copy(int64_t n, const float *in, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
