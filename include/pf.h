/*
 * pf.h -- C ABI of the MI355X (gfx950) clamp-to-edge image filter library
 * (libpencilfilter.so).
 *
 * Shape of every call, after the paper's coding rules for a PENCIL function
 * (Sec. II-B.1): sizes come first, then arrays declared as C99 VLAs qualified
 * `restrict const static` (distinct arrays never overlap, each holds at least
 * the stated number of elements), then scalar out-parameters as
 * `T *const restrict`. Batches are described without arrays of pointers: one
 * arena per kind of data plus per-item offsets, the (array, index) form the
 * paper gives for OP2's rewritten kernel (Sec. III-A). Semantics are those of
 * the sequential loop nest, whose output iterations are independent
 * (Sec. II-B.3), so the library computes them in any order.
 *
 * Filter semantics (all entry points): correlation without kernel flip,
 *     out[y][x] = sum_{dy=-r..r} sum_{dx=-r..r} f[dy+r][dx+r] * in[cy][cx],
 *     cy = clamp(y+dy, 0, h-1),  cx = clamp(x+dx, 0, w-1)
 * with row-major dense images (pitch = w) and row-major filters. The
 * separable form computes the row pass with fx (horizontal taps) into an
 * FP32 intermediate and then the column pass with fy (vertical taps).
 *
 * Memory: unless stated otherwise, every array argument is a DEVICE pointer
 * (HIP device memory of the current device, e.g. a torch tensor's
 * data_ptr()). `stream` is a hipStream_t passed as void*; NULL is the null
 * stream. The caller owns every buffer it passes. Filter calls are
 * asynchronous on `stream`: they return after enqueueing, and their buffers
 * must stay alive and unmodified until the stream reaches the work. The
 * library keeps no pointer to caller memory after the call returns (batch
 * plans keep none beyond a run either).
 *
 * Errors: no exception crosses the ABI. Every call returns a pf_status;
 * pf_last_error() gives a thread-local message for the last failing call on
 * the calling thread. Arguments are validated before anything is enqueued;
 * an invalid call enqueues nothing. Asynchronous device faults surface on a
 * later synchronising call as PF_EDEVICE.
 *
 * Precision: FP32 results agree with the sequential definition within the
 * FP32 inner-product bound (taps may be fused multiply-adds, summed in the
 * definition's order dy outer, dx inner). With PF_FLAG_EXACT the FP32 paths
 * use a separate multiply and add per tap in that same order, and reproduce
 * the sequential C program bit for bit. The integer path is exact.
 */
#ifndef PENCILFILTER_PF_H
#define PENCILFILTER_PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
/* C++ sees each VLA parameter as a restrict-qualified pointer. */
#define PF_ARR(T, name, n) T *__restrict name
#define PF_OUTP(T, name) T *const __restrict name
#else
#define PF_ARR(T, name, n) T name[restrict const static (n)]
#define PF_OUTP(T, name) T *const restrict name
#endif

/* ---- status ------------------------------------------------------------- */
typedef int32_t pf_status;
#define PF_OK            0  /* success                                        */
#define PF_EINVAL        1  /* bad size, radius, null pointer, bad flag       */
#define PF_EALIAS        2  /* input and output ranges overlap (restrict)     */
#define PF_EUNSUPPORTED  3  /* valid C, but outside what this build supports */
#define PF_EDEVICE       4  /* HIP runtime or device error                    */
#define PF_ENOMEM        5  /* host or device allocation failed               */
#define PF_EBUDGET       6  /* request larger than the whole HBM budget       */
#define PF_EAGAIN        7  /* queue full or result not ready; try again      */
#define PF_ETIMEDOUT     8  /* wait ended before completion                   */

/* Largest supported filter radius (filters up to 17 x 17). */
#define PF_R_MAX 8
/* Largest radius inside batch plans and served requests (9 x 9 filters):
 * the persistent batch kernel is built only for radii 0..4, where every
 * body fits in registers; larger radii run as single-image calls. */
#define PF_BATCH_R_MAX 4

/* Flags for single-image calls, batch plans and servers. */
#define PF_FLAG_EXACT       0x1  /* separate FP32 mul and add per tap, definition order */
#define PF_BATCH_GRAPH      0x2  /* batch plan: capture its launches in a hipGraph      */
#define PF_BATCH_NO_TUNE    0x4  /* batch plan: ignore the tune table, use defaults     */

/* Filter kinds inside a batch or a served request (and tune-table keys). */
#define PF_KIND_2D   0  /* (2r+1)^2 weights, row-major, at filt_off               */
#define PF_KIND_SEP  1  /* fx[2r+1] at filt_off, then fy[2r+1] right after it     */
#define PF_KIND_U8   2  /* tune-table key of the uint8 path (not a batch kind)    */

/* Execution variants a kind may run as (chosen by the tune table). */
#define PF_VAR_DIRECT      0  /* full 2D taps                                     */
#define PF_VAR_SEPARABLE   1  /* fused row pass + column pass (PF_KIND_SEP only)  */
#define PF_VAR_SEP_DIRECT  2  /* PF_KIND_SEP run as 2D taps fy[i]*fx[j] (FP32)    */
/* Largest radius PF_VAR_SEP_DIRECT runs at: above it the (2r+1)^2 computed
 * taps no longer fit in registers (PF_EUNSUPPORTED). */
#define PF_SEP_DIRECT_R_MAX 5
/* PF_KIND_U8 on the int8 matrix cores (v_mfma_i32_16x16x64_i8) instead of
 * v_dot4, radius 1..PF_U8_MFMA_R_MAX; same results bit for bit. Its launch
 * shape: rows_per_wave a multiple of 16, rows_per_wave * waves_per_group
 * at most PF_U8_MFMA_TILE_MAX (the rows of a workgroup tile of 128 columns). */
#define PF_VAR_MFMA        3
#define PF_U8_MFMA_R_MAX   8
#define PF_U8_MFMA_TILE_MAX 256

/* Border rules: the value an index outside [0, n) of an axis reads. */
#define PF_BORDER_CLAMP    0  /* nearest edge element: a a | a b c | c c           */
#define PF_BORDER_ZERO     1  /* zero                                              */
#define PF_BORDER_REFLECT  2  /* edge repeated, period 2n: b a | a b c | c b       */
#define PF_BORDER_MIRROR   3  /* edge not repeated, period 2n-2: c b | a b c | b a  */

/* Largest r * passes of a filter chain (the halo one LDS tile carries). */
#define PF_CHAIN_HALO_MAX 16

const char *pf_status_str(pf_status s);
/* Message of the last failing call on this thread ("" if none). The string
 * stays valid until the next pf_* call on the same thread. */
const char *pf_last_error(void);
/* Library version string, and the gfx target the kernels were built for. */
const char *pf_version(void);

/* ---- single image: FP32 full 2D -----------------------------------------
 * Sec. II (stencils as regular, statically analysable loop nests) and
 * Sec. II-B.1 (calling convention). h, w >= 1; 0 <= r <= PF_R_MAX.
 * in, out: float[h*w] device, 4-byte aligned, disjoint (else PF_EALIAS).
 * filt: float[(2r+1)^2] device. flags: 0 or PF_FLAG_EXACT. */
pf_status pf_filter2d_f32(int32_t h, int32_t w, int32_t r,
                          PF_ARR(const float, in, h * w),
                          PF_ARR(const float, filt, (2 * r + 1) * (2 * r + 1)),
                          PF_ARR(float, out, h * w),
                          int32_t flags, void *stream);

/* ---- single image: FP32 full 2D under a border rule ---------------------
 * As pf_filter2d_f32, with the image extended past its edges by `border`
 * (PF_BORDER_*); each axis is mapped on its own, so a corner reads the
 * element both mappings select. Stencil codes of the image-processing and
 * fluid-dynamics domains (Sec. I) use all four rules. PF_BORDER_CLAMP runs
 * the same kernel as pf_filter2d_f32; the other rules run the chain kernel
 * with one pass (r * 1 <= PF_CHAIN_HALO_MAX). Unknown rule: PF_EINVAL. */
pf_status pf_filter2d_f32_border(int32_t h, int32_t w, int32_t r, int32_t border,
                                 PF_ARR(const float, in, h * w),
                                 PF_ARR(const float, filt, (2 * r + 1) * (2 * r + 1)),
                                 PF_ARR(float, out, h * w),
                                 int32_t flags, void *stream);

/* ---- single image: chain of FP32 2D passes, fused ------------------------
 * `passes` >= 1 applications of the same filter: pass p filters the FP32
 * image of pass p-1 (the input for p = 1) extended by `border`, and `out`
 * receives the last. All passes run in one kernel over LDS tiles that carry
 * a halo of r * passes (<= PF_CHAIN_HALO_MAX, else PF_EUNSUPPORTED): the
 * intermediate images never reach HBM. This is the composition of stencil
 * kernels that cross-component optimisation targets (Sec. II). With
 * PF_FLAG_EXACT every pass is the sequential definition bit for bit; by
 * default each tap is one fused multiply-add. Same buffer rules as
 * pf_filter2d_f32. */
pf_status pf_filter_chain_f32(int32_t h, int32_t w, int32_t r, int32_t passes, int32_t border,
                              PF_ARR(const float, in, h * w),
                              PF_ARR(const float, filt, (2 * r + 1) * (2 * r + 1)),
                              PF_ARR(float, out, h * w),
                              int32_t flags, void *stream);

/* ---- reductions: sum and mean of an FP32 array ---------------------------
 * The `reduction` directive (Sec. II-B.3) and OptiML's sum lowered to a
 * loop with a reduction (Sec. III-B). out[0] = sum of x[0..n) and out[1] =
 * out[0] / n, in float64. Reproducible (Sec. III-A's concern): a fixed
 * summation tree, the same bits on every call and launch. n >= 1, at most
 * 2^40. x: float[n] device, 4-byte aligned. out: double[2] device, 8-byte
 * aligned. workspace: device memory of at least pf_sum_workspace(n) bytes,
 * 8-byte aligned, owned by the caller, no initial contents needed; calls
 * sharing one workspace must not overlap in time. Overlap between x, out
 * and workspace: PF_EALIAS. Two launches on `stream`, no allocation. */
pf_status pf_sum_workspace(int64_t n, PF_OUTP(size_t, bytes));
pf_status pf_sum_f32(int64_t n, PF_ARR(const float, x, n), PF_ARR(double, out, 2),
                     void *workspace, size_t workspace_bytes, void *stream);

/* ---- reductions: sum and mean without any allocation --------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and the same bits as pf_sum_f32, with the chunk partials in a
 * static device array of the library (64 KiB on each GPU it runs on, held
 * until the process ends) instead of a caller workspace. n >= 1 and at most
 * 2^29 (8192 chunks of 65536 elements; larger n: PF_EUNSUPPORTED). x:
 * float[n] device, 4-byte aligned; out: double[2] device, 8-byte aligned;
 * x and out disjoint (else PF_EALIAS). Two launches on `stream`; calls no
 * hipMalloc, hipFree or allocating library routine. Every call on one GPU
 * shares that GPU's scratch, so calls that overlap in time on one GPU (on
 * different streams, or from several threads) race and must be ordered by
 * the caller; nothing in the scratch needs to start at zero. */
pf_status pf_sum_f32_noalloc(int64_t n, PF_ARR(const float, x, n), PF_ARR(double, out, 2), void *stream);

/* ---- reductions: 256-bin histogram of a uint8 array ----------------------
 * The indirect increment A[t[i]]++ of the `independent` example
 * (Sec. II-B.3) with repeated indices: hist[v] = number of i with
 * x[i] == v. Exact. n >= 1, at most 2^40. x: uint8_t[n] device (any
 * alignment). hist: int64_t[256] device, 8-byte aligned. workspace: at
 * least pf_hist_workspace(n) bytes, 4-byte aligned, as for pf_sum_f32. */
pf_status pf_hist_workspace(int64_t n, PF_OUTP(size_t, bytes));
pf_status pf_hist256_u8(int64_t n, PF_ARR(const uint8_t, x, n), PF_ARR(int64_t, hist, 256),
                        void *workspace, size_t workspace_bytes, void *stream);

/* ---- OP2 indirect increment: edges add into cells -----------------------
 * OP2's op_par_loop over edges with two OP_INC arguments through an
 * edge-to-cell map (Sec. III-A): for i = 0 .. nedges-1 in order,
 * cell[map[2i+1]] += edge[i], then cell[map[2i]] += edge[i] (float64).
 *
 * Plan path (reproducible, equal to that loop bit for bit): the plan
 * inverts the map once (host copy `edge_to_cells`, int32[2 * nedges],
 * read during the call only; entries in 0..ncells-1, else PF_EINVAL;
 * nedges <= 2^30) and keeps its tables in device memory until destroyed.
 * pf_inc_plan_run adds every cell's increments in the loop's order, one
 * thread per cell: edge: double[nedges] device, cell: double[ncells]
 * device (read and written), 8-byte aligned, disjoint (else PF_EALIAS);
 * sizes must match the plan's. */
typedef struct pf_inc_plan pf_inc_plan;
pf_status pf_inc_plan_create(int32_t ncells, int32_t nedges,
                             PF_ARR(const int32_t, edge_to_cells, 2 * nedges),
                             PF_OUTP(pf_inc_plan *, plan));
pf_status pf_inc_plan_run(const pf_inc_plan *plan, int32_t ncells, int32_t nedges,
                          PF_ARR(const double, edge, nedges), PF_ARR(double, cell, ncells),
                          void *stream);
pf_status pf_inc_plan_destroy(pf_inc_plan *plan);

/* Atomic path: one launch, float64 atomic adds, no plan. The map is a
 * device array (int32[2 * nedges], 4-byte aligned); entries outside
 * 0..ncells-1 are skipped. The order of a cell's increments varies from
 * run to run, so results agree with the loop only to rounding. */
pf_status pf_edge_inc_atomic_f64(int32_t ncells, int32_t nedges,
                                 PF_ARR(const int32_t, edge_to_cells, 2 * nedges),
                                 PF_ARR(const double, edge, nedges), PF_ARR(double, cell, ncells),
                                 void *stream);

/* ---- single image: FP32 separable ---------------------------------------
 * Row pass with fx, FP32 intermediate, column pass with fy, fused in one
 * kernel: the intermediate never reaches memory (the cross-kernel fusion
 * that Sec. II's cross-component optimisation motivates). Same rules as
 * pf_filter2d_f32; fx and fy: float[2r+1] device. */
pf_status pf_filter_sep_f32(int32_t h, int32_t w, int32_t r,
                            PF_ARR(const float, in, h * w),
                            PF_ARR(const float, fx, 2 * r + 1),
                            PF_ARR(const float, fy, 2 * r + 1),
                            PF_ARR(float, out, h * w),
                            int32_t flags, void *stream);

/* ---- single image: uint8 planar, integer ----------------------------------
 * The same stencil loop nest (Sec. II, stencils as regular algorithms; the
 * image-processing domain of Sec. I) in integer arithmetic, with the
 * calling convention of Sec. II-B.1. c planes of h x w uint8 (plane p at
 * offset p*h*w), one int8 filter for all planes: acc = sum of int8 weight * uint8 pixel in int32 (exact),
 * q = acc >> shift (arithmetic, i.e. floor), out = min(max(q, 0), 255).
 * c, h, w >= 1; 0 <= r <= PF_R_MAX; 0 <= shift <= 31. in and out disjoint.
 * filt: int8[(2r+1)^2] device. flags must be 0. The tune table's variant
 * picks the kernel: PF_VAR_MFMA (the int8 matrix cores; radii 1..8, the
 * default there) or PF_VAR_DIRECT (v_dot4, every radius); both give the
 * same bytes. For v_dot4 the table's tile height is the tallest tile: the
 * launch keeps the number of rounds of waves per SIMD that height needs
 * and spreads each strip column's rows evenly over as many tiles as fill
 * those rounds (integer sums, so the result does not depend on the split). */
pf_status pf_filter2d_u8(int32_t c, int32_t h, int32_t w, int32_t r, int32_t shift,
                         PF_ARR(const uint8_t, in, c * h * w),
                         PF_ARR(const int8_t, filt, (2 * r + 1) * (2 * r + 1)),
                         PF_ARR(uint8_t, out, c * h * w),
                         int32_t flags, void *stream);

/* ---- single image with an explicit launch shape ----------------------------
 * The same computation as the call for `kind`/`variant`, with the launch
 * shape forced: rows_per_wave a multiple of 4 in 4..128, waves_per_group in
 * {1, 2, 4, 8}. Used by the autotuner and by tests that check results do
 * not depend on the launch shape. kind PF_KIND_2D requires variant
 * PF_VAR_DIRECT; PF_KIND_SEP accepts all three variants. For PF_KIND_SEP,
 * filt holds fx then fy (2*(2r+1) floats). */
pf_status pf_filter_f32_shaped(int32_t h, int32_t w, int32_t r, int32_t kind, int32_t variant,
                               int32_t rows_per_wave, int32_t waves_per_group,
                               PF_ARR(const float, in, h * w),
                               const float *filt,
                               PF_ARR(float, out, h * w),
                               int32_t flags, void *stream);

/* ---- tuning (profile-based auto-tuning, Sec. II, Fig. 1 flow) -------------
 * The tune table maps (context, kind, r, size class) to a variant and a
 * launch shape. Contexts: PF_TUNE_SINGLE for single-image calls,
 * PF_TUNE_BATCH for the persistent batch kernel of batch plans and servers
 * (FP32 kinds only; four waves per workgroup; direct or separable
 * variant). Size classes: 0 small (< 256*256 px), 1 medium, 2 large
 * (> 1024*1024 px). A built-in default table is used until one is loaded.
 * Results depend on the variant only, never on the launch shape. */
#define PF_TUNE_SINGLE 0
#define PF_TUNE_BATCH  1

typedef struct pf_tune_entry {
    int32_t kind;             /* PF_KIND_2D, PF_KIND_SEP, PF_KIND_U8 */
    int32_t r;                /* 0..PF_R_MAX                   */
    int32_t size_class;       /* 0, 1, 2                       */
    int32_t variant;          /* PF_VAR_*                      */
    int32_t rows_per_wave;
    int32_t waves_per_group;
    float   us;               /* measured median time of the winning candidate (us), or 0:
                                 one launch of the class image (PF_TUNE_SINGLE), one batch
                                 launch of class images (PF_TUNE_BATCH, pf_autotune) or of
                                 the whole tuned batch (PF_TUNE_BATCH, pf_batch_autotune) */
    int32_t context;          /* PF_TUNE_SINGLE or PF_TUNE_BATCH */
} pf_tune_entry;

pf_status pf_tune_lookup(int32_t kind, int32_t r, int64_t pixels, int32_t context, PF_OUTP(pf_tune_entry, e));
/* Replace the active table with n entries (missing keys keep defaults). */
pf_status pf_tune_set(int32_t n, PF_ARR(const pf_tune_entry, entries, n));
pf_status pf_tune_reset(void);
/* Load / save the table as JSON text (host file path). */
pf_status pf_tune_load(const char *path);
pf_status pf_tune_save(const char *path);
/* Measure, on the current device with hipEvents (median of 5 groups of
 * `reps` timed runs over buffers rotated through 1 GiB), for r in 0..r_max
 * and the three size
 * classes: every (rows_per_wave in {8, 16, 32, 64}, for PF_KIND_U8 also
 * 12, 20, 24 and 48, for the FP32 kinds also the heights up to 64 that fill
 * whole row chunks of the radius) x (waves_per_group in {1, 2, 4, 8}) shape of
 * single-image calls of every kind, and for
 * PF_KIND_SEP (r <= PF_SEP_DIRECT_R_MAX) also the PF_VAR_SEP_DIRECT variant
 * at the best shape, and for PF_KIND_U8 (r <= PF_U8_MFMA_R_MAX) also the
 * PF_VAR_MFMA variant at rows_per_wave in {16, 32, 48, 64} x
 * waves_per_group in {1, 2, 4, 8} within PF_U8_MFMA_TILE_MAX; and the
 * tile heights {8, 16, 32, 64} of the batch kernel on a batch of class
 * images (FP32 kinds). A candidate replaces the default only when at least
 * 3% faster. Installs the winners and writes the table to `path` if it is
 * not NULL. Allocates and frees its own device buffers; synchronises the
 * device. */
pf_status pf_autotune(int32_t r_max, int32_t reps, const char *path);
/* Workgroups (of four waves) per compute unit that persistent batch
 * launches use, a table-wide setting (saved with the table; reset to its
 * default, 1, by pf_tune_set and pf_tune_reset). `blocks_per_cu` in 1..8
 * sets it, 0 leaves it; the value before the call goes to `previous` if
 * not NULL. Fewer than fit at once is deliberate: on MI355X the fewest
 * tiles in flight ran fastest. Plans created earlier keep their grid. */
pf_status pf_tune_batch_blocks(int32_t blocks_per_cu, int32_t *previous);
/* Tune the PF_TUNE_BATCH entries for one batch (the arguments of
 * pf_batch_plan_create and pf_batch_plan_run), timing whole-batch launches
 * on the device (median of 5 x `reps`): first a joint grid of workgroups
 * per compute unit (1..4, see pf_tune_batch_blocks) x one row-tile height
 * in {8, 16, 32, 64} for every key the batch uses, keeping the fastest
 * point; then for each (kind, r, size class) key the batch uses, the other
 * tile heights of that set and those up to 64 that fill whole row chunks of
 * the key's radius, keeping a change only when the batch gets at least 3%
 * faster. Single-image entries are not touched. Installs the result and
 * writes it to `path` if not NULL. Overwrites `out`. */
pf_status pf_batch_autotune(int32_t n,
                            PF_ARR(const int32_t, h, n), PF_ARR(const int32_t, w, n),
                            PF_ARR(const int32_t, r, n), PF_ARR(const int32_t, kind, n),
                            PF_ARR(const int64_t, pix_off, n), PF_ARR(const int64_t, filt_off, n),
                            int64_t npix, int64_t nfilt,
                            PF_ARR(const float, in, npix), PF_ARR(const float, filt, nfilt),
                            PF_ARR(float, out, npix), int32_t reps, const char *path);

/* ---- batch: many images, one persistent launch ---------------------------
 * Arrays plus per-item offsets instead of arrays of pointers, the form the
 * paper gives OP2's rewritten kernel (Sec. III-A); every output element of
 * every image is an independent iteration (Sec. II-B.3), so all images'
 * tiles run in one launch. Radii 0..PF_BATCH_R_MAX (else PF_EUNSUPPORTED).
 * n images described by host arrays (sizes first): image i has h[i] x w[i]
 * pixels at in + pix_off[i] and out + pix_off[i], radius r[i], filter kind
 * kind[i] with weights at filt + filt_off[i]. Offsets are in elements.
 * Plan creation validates everything (ranges inside npix / nfilt, images
 * disjoint), chooses each image's variant and shape from the tune table,
 * builds the tile table and uploads it to the device. The plan owns that
 * device table (and, with PF_BATCH_GRAPH, a captured hipGraph).
 * Variant choice depends only on (kind, r, pixels), never on the rest of
 * the batch, so each image's result equals what the single-image call with
 * the same variant computes, bit for bit. */
typedef struct pf_batch_plan pf_batch_plan;

pf_status pf_batch_plan_create(int32_t n,
                               PF_ARR(const int32_t, h, n), PF_ARR(const int32_t, w, n),
                               PF_ARR(const int32_t, r, n), PF_ARR(const int32_t, kind, n),
                               PF_ARR(const int64_t, pix_off, n), PF_ARR(const int64_t, filt_off, n),
                               int64_t npix, int64_t nfilt, int32_t flags,
                               PF_OUTP(pf_batch_plan *, plan));
/* Run the plan: in, out: float[npix] device arenas (disjoint); filt:
 * float[nfilt] device arena. npix and nfilt must equal the plan's. With
 * PF_BATCH_GRAPH the launch is a graph replay; new arena pointers are
 * patched into the graph's kernel nodes before the replay. */
pf_status pf_batch_plan_run(pf_batch_plan *plan, int64_t npix, int64_t nfilt,
                            PF_ARR(const float, in, npix), PF_ARR(const float, filt, nfilt),
                            PF_ARR(float, out, npix), void *stream);
/* Per-image variant chosen by the plan (host array of n entries). */
pf_status pf_batch_plan_variants(const pf_batch_plan *plan, int32_t n, PF_ARR(int32_t, variant, n));
/* tasks: wave tiles in the plan; launches: kernels per run (1 or 2);
 * grid: workgroups of the main persistent launch. */
pf_status pf_batch_plan_info(const pf_batch_plan *plan, PF_OUTP(int64_t, tasks),
                             PF_OUTP(int32_t, launches), PF_OUTP(int32_t, grid));
pf_status pf_batch_plan_destroy(pf_batch_plan *plan);

/* ---- serving: continuous batching under an HBM budget ----------------------
 * Independent calls (Sec. II-B.3) arriving over time share batches: the
 * filter requests of a batch run in one persistent launch (the batch form
 * above), its reductions (the `reduction` directive, Sec. II-B.3; OptiML's
 * sum, Sec. III-B) in the multi-array sum and histogram kernels.
 * A server owns a device arena of `hbm_budget_bytes` (results, uploaded
 * inputs), `n_streams` HIP streams with their descriptor and workspace
 * buffers (allocated at creation) and an engine thread. Requests are
 * admitted first-come first-served while their bytes fit in the budget;
 * admitted requests are packed into batches of at most `max_batch` requests
 * and launched on whichever stream is free, so new arrivals run while
 * earlier batches are still on the device. While another batch is running,
 * a launch waits up to 50 us (from its oldest request's arrival) for at
 * least max_batch/2 admitted requests; with the device idle a request
 * launches at once. A request's result does not
 * depend on which batch it lands in: filters as the single-image call with
 * the same variant, sums and histograms bit for bit as pf_sum_f32 and
 * pf_hist256_u8. Served filter radii: 0..PF_BATCH_R_MAX. */
typedef struct pf_server pf_server;

typedef struct pf_server_stats {
    int64_t submitted, admitted, completed, rejected;
    int64_t batches;              /* batches launched                          */
    int64_t pixels;               /* output pixels completed                   */
    int64_t bytes_high_water;     /* largest arena reservation seen            */
    int64_t queue_high_water;     /* largest number of waiting requests        */
    double  mean_batch;           /* requests per batch                        */
    double  p50_us, p99_us, p999_us, max_us;   /* completion - arrival         */
    double  wall_s;               /* first arrival to last completion          */
    double  gpx_per_s;            /* pixels / wall_s / 1e9                     */
} pf_server_stats;

/* n_streams 1..8, max_batch 1..4096, max_queue >= 1 (waiting requests).
 * flags: 0 or PF_FLAG_EXACT (filters in the bit-reproducible mode). */
pf_status pf_server_create(int64_t hbm_budget_bytes, int32_t n_streams, int32_t max_batch,
                           int32_t max_queue, int32_t flags, PF_OUTP(pf_server *, srv));
/* Submit one filter request (sizes first). `in` is float[h*w]: a device
 * pointer that stays allocated and unmodified until the request completes,
 * or, if in_is_host != 0, a host pointer copied before submit returns.
 * For a device input, `stream` (a hipStream_t; NULL is the null stream) is
 * the stream whose queued work produces `in`: the server's launch waits for
 * the work queued there at submit time. `filt` is a HOST array of the
 * kind's weights, copied. The arrival time (ns on CLOCK_MONOTONIC; 0 = now)
 * is the origin of the request's latency. PF_EBUDGET if the request alone
 * exceeds the budget, PF_EAGAIN if max_queue requests are already waiting,
 * PF_EUNSUPPORTED for r > PF_BATCH_R_MAX. */
pf_status pf_server_submit(pf_server *s, int32_t h, int32_t w, int32_t r, int32_t kind,
                           const float *in, int32_t in_is_host,
                           const float *filt, void *stream, int64_t arrival_ns,
                           PF_OUTP(int64_t, ticket));
/* Reductions served beside the filters. */
#define PF_OP_SUM_F32  1   /* sum and mean of float[n]: result double[2]      */
#define PF_OP_HIST_U8  2   /* 256-bin histogram of uint8_t[n]: int64_t[256]   */
/* Submit one reduction of n elements (1 <= n <= 2^40): `in` as for
 * pf_server_submit (device pointer ordered after `stream`, 4-byte aligned
 * for PF_OP_SUM_F32; or host memory, copied). Same statuses as
 * pf_server_submit. */
pf_status pf_server_submit_reduce(pf_server *s, int32_t op, int64_t n, const void *in, int32_t in_is_host,
                                  void *stream, int64_t arrival_ns, PF_OUTP(int64_t, ticket));
/* done = 1 once the request's output is complete on the device. */
pf_status pf_server_poll(pf_server *s, int64_t ticket, PF_OUTP(int32_t, done));
/* Block until done or timeout (ns; < 0 waits forever): PF_ETIMEDOUT. */
pf_status pf_server_wait(pf_server *s, int64_t ticket, int64_t timeout_ns);
/* Copy the finished output (float[h*w]) to `out` (host if out_is_host,
 * else device) and release the request's arena bytes and ticket. */
pf_status pf_server_result(pf_server *s, int64_t ticket, int32_t h, int32_t w,
                           float *out, int32_t out_is_host);
/* Copy a finished reduction's result (double[2] for PF_OP_SUM_F32,
 * int64_t[256] for PF_OP_HIST_U8; host if out_is_host, else device) and
 * release it. `op` must be the request's. */
pf_status pf_server_result_reduce(pf_server *s, int64_t ticket, int32_t op, void *out, int32_t out_is_host);
/* Release a finished request without copying its output. */
pf_status pf_server_release(pf_server *s, int64_t ticket);
pf_status pf_server_stats_get(pf_server *s, PF_OUTP(pf_server_stats, st));
/* Open-loop load generator (filter requests only): submit n requests at
 * their scheduled times
 * (arrival_ns[i], relative to the call's start), request i filtering
 * h[i] x w[i] pixels at in + pix_off[i] (device arena of npix floats) with
 * radius r[i] and host weights filt + filt_off[i] (kind PF_KIND_SEP), and
 * release each output as it completes. The pool must be complete (no work
 * producing it still queued) when the call starts. Returns when all have
 * completed; latencies are recorded in the server's stats. */
pf_status pf_server_run_trace(pf_server *s, int32_t n,
                              PF_ARR(const int64_t, arrival_ns, n),
                              PF_ARR(const int32_t, h, n), PF_ARR(const int32_t, w, n),
                              PF_ARR(const int32_t, r, n),
                              PF_ARR(const int64_t, pix_off, n), PF_ARR(const int64_t, filt_off, n),
                              int64_t npix, const float *in, int64_t nfilt, const float *filt);
/* Stop: requests not yet admitted fail (PF_EAGAIN from wait/poll while the
 * server exists), admitted ones run to completion; then free everything the
 * server owns. No call on `s` may run concurrently with or after it. */
pf_status pf_server_destroy(pf_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PENCILFILTER_PF_H */
