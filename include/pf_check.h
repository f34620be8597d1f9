/*
 * pf_check.h -- host-side diagnostics of libpencilfilter.so.
 *
 * Calls here touch no device: they run on any host, with or without a GPU,
 * and exist so that the library's own tables can be checked on the CPU.
 * Conventions (status codes, thread-local message, PF_ARR / PF_OUTP) are
 * those of pf.h.
 */
#ifndef PENCILFILTER_PF_CHECK_H
#define PENCILFILTER_PF_CHECK_H

#include "pf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Builds the host tables that pf_batch_plan_create would build for the same
 * arguments (same validation, same status on invalid input; tile heights
 * from the batch context of the active tune table) and replays on the host
 * where every wave tile of the persistent batch kernel reads and writes,
 * with the strip-geometry functions the kernel itself uses: every tile must
 * name a valid image, a strip and row band inside it, and every vector
 * load, halo load and unguarded vector store of each of its 64 lanes must
 * fall inside its image row; every image must lie inside the pixel arena.
 * Batches are the arena-plus-offsets description of Sec. III-A; the check
 * is that each tile's accesses stay within its image's span of the arena.
 * tiles: number of wave tiles checked; violations: number found (PF_EINVAL
 * with the first described in pf_last_error() when > 0). */
pf_status pf_batch_plan_check(int32_t n,
                              PF_ARR(const int32_t, h, n), PF_ARR(const int32_t, w, n),
                              PF_ARR(const int32_t, r, n), PF_ARR(const int32_t, kind, n),
                              PF_ARR(const int64_t, pix_off, n), PF_ARR(const int64_t, filt_off, n),
                              int64_t npix, int64_t nfilt, int32_t flags,
                              PF_OUTP(int64_t, tiles), PF_OUTP(int64_t, violations));

/* Replays operations on the first-fit allocator that a server uses for its
 * HBM arena (host bookkeeping only; no device memory is touched): op[i] > 0
 * allocates op[i] bytes (rounded up to 256), op[i] < 0 frees the allocation
 * made by operation -op[i] - 1. result[i] is the allocation's offset, or -1
 * if no free run was large enough; 0 for a free. A free of an operation
 * that was not a successful, still live allocation: PF_EINVAL. used: the
 * bytes allocated after the last operation. */
pf_status pf_arena_replay(int64_t budget, int32_t n, PF_ARR(const int64_t, op, n), PF_ARR(int64_t, result, n),
                          PF_OUTP(int64_t, used));

#ifdef __cplusplus
}
#endif

#endif /* PENCILFILTER_PF_CHECK_H */
