// Internal declarations shared by the library's translation units.
// Nothing here is part of the C ABI (that is include/pf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include <vector>

#include "pf.h"
#include "pf_check.h"

namespace pf {

// A wave strip is 64 lanes x 4 columns. halo_lanes: neighbouring lanes on
// each side whose columns a lane's window needs. For radii 1 and 2 every
// lane produces outputs (256 columns, 1 KiB of FP32) and lanes 0 and 63
// also load the r columns beyond the strip (r registers per row); for
// larger radii, where those registers would cost occupancy, the outermost
// lanes only load halo columns and do not store.
#ifndef PF_STRIP_ALIGNED
#define PF_STRIP_ALIGNED 1
#endif
#ifndef PF_STRIP_ALIGNED_RMAX
#define PF_STRIP_ALIGNED_RMAX 2
#endif
constexpr int halo_lanes(int r) { return (r + 3) / 4; }
constexpr bool aligned_strip(int r) { return PF_STRIP_ALIGNED && r >= 1 && r <= PF_STRIP_ALIGNED_RMAX; }
constexpr int idle_lanes(int r) { return aligned_strip(r) ? 0 : halo_lanes(r); }
constexpr int strip_width(int r) { return 4 * (64 - 2 * idle_lanes(r)); }
// The uint8 strip keeps its halo lanes at every radius.
constexpr int strip_width_u8(int r) { return 4 * (64 - 2 * halo_lanes(r)); }

// ---- strip geometry, shared by the FP32 strip kernels and the host-side
// check of batch plans (constexpr functions compile for host and device).

// How a strip loads its rows (uniform over the wave):
//   kStripFast: every lane's 4 columns lie inside the image (a halo lane
//               left of column 0 aside): one 16-byte load per lane;
//   kStripEdge: some columns lie outside; the lane loads the 4 in-bounds
//               columns nearest to its own (w >= 4) and picks each clamped
//               column from them;
//   kStripTiny: one clamped load per column (images narrower than 4
//               columns, and every strip of radii above 4).
constexpr int kStripFast = 0, kStripEdge = 1, kStripTiny = 2;

// Rows per pipelined chunk of the FP32 strip: a multiple of K = 2r+1 (ring
// residues stay compile-time constants) near `chunk` rows. Single-image
// launches take 8, the persistent batch kernel 12 (both measured on
// MI355X). Rows past the last whole chunk of a tile are taken in groups of
// 2r+1 with a wait per group, so tile heights that fill whole chunks skip
// that tail (the tuners try them).
#ifndef PF_CHUNK
#define PF_CHUNK 8
#endif
#ifndef PF_BATCH_CHUNK
#define PF_BATCH_CHUNK 12
#endif
constexpr int chunk_rows_of(int r, int chunk) {
    return (2 * r + 1) * (chunk / (2 * r + 1) > 0 ? chunk / (2 * r + 1) : 1);
}

constexpr int clamp_int(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// First column of lane `lane` in a strip starting at column x0.
constexpr int lane_col(int r, int x0, int lane) { return x0 + 4 * (lane - idle_lanes(r)); }

// kStripFast needs every lane's columns to end inside the image; for an
// aligned strip also the r columns to its right inside it, or none.
constexpr bool fast_strip(int r, int x0, int w) {
    const int end = x0 + 4 * (64 - idle_lanes(r));
    return aligned_strip(r) ? (end <= w && (end == w || end + r <= w)) : end <= w;
}

constexpr int strip_mode(int r, int x0, int w) {
    return r > 4 ? kStripTiny : (fast_strip(r, x0, w) ? kStripFast : (w >= 4 ? kStripEdge : kStripTiny));
}

// First of the 4 columns the 16-byte load of a lane with first column xs
// reads in kStripFast and kStripEdge (a halo lane left of column 0 reads
// columns 0..3).
constexpr int vec_load_col(int r, int mode, int xs, int w) {
    return mode == kStripFast ? (idle_lanes(r) > 0 ? (xs > 0 ? xs : 0) : xs) : clamp_int(xs, 0, w - 4);
}

// First of the r columns the halo load of an aligned strip reads in
// kStripFast: left of the strip (lanes 0..31) or right of it (lanes 32..63),
// moved inside the image at its edges.
constexpr int halo_load_col(int r, bool left, int x0, int w) {
    return left ? (x0 - r > 0 ? x0 - r : 0) : (x0 + 4 * 64 < w - r ? x0 + 4 * 64 : w - r);
}

// Order of the FP32 kernels' wave tiles inside an image: row-major over the
// image's strips (0) or column-major (1).
#ifndef PF_TILE_COLMAJOR
#define PF_TILE_COLMAJOR 0
#endif
constexpr bool kTileColMajorF32 = PF_TILE_COLMAJOR != 0;

// Tile number -> (strip x, strip y): row-major over the image's strips, or
// column-major (strip by strip down the image).
constexpr void tile_strip(bool colmajor, int t, int strips_x, int strips_y, int &sx, int &sy) {
    if (colmajor) {
        sx = t / strips_y;
        sy = t - sx * strips_y;
    } else {
        sy = t / strips_x;
        sx = t - sy * strips_x;
    }
}

// One image of a batch as the persistent kernel sees it. `var` is the
// executed variant (PF_VAR_*), `by` rows per wave tile; the image's wave
// tiles are numbered column-major over (strip x, strip y).
// Element offsets are added to the kernel's base pointers as integers, so a
// descriptor may also carry an absolute address (byte address / 4) with a
// null base.
struct BatchImg {
    int64_t in_off;
    int64_t out_off;
    int64_t filt_off;
    int32_t h, w, r, var;
    int32_t by, strips_x, strips_y, pad;
};

// One entry of a wave's tile list: the image (index into the descriptor
// array) and the tile's number inside the image.
struct BatchTask {
    int32_t img, tile;
};

// Fills strips_x and strips_y of a descriptor whose r, h, w and by are set;
// returns its wave-tile count.
inline int64_t set_strips(BatchImg &d) {
    d.strips_x = (d.w + strip_width(d.r) - 1) / strip_width(d.r);
    d.strips_y = (d.h + d.by - 1) / d.by;
    d.pad = 0;
    return (int64_t)d.strips_x * d.strips_y;
}

// Appends the wave tiles of image `img` (descriptor d) to a batch's tile list.
inline void append_tiles(std::vector<BatchTask> &list, int32_t img, const BatchImg &d) {
    const int32_t n = d.strips_x * d.strips_y;
    for (int32_t t = 0; t < n; ++t) list.push_back({img, t});
}

// Host tables of a batch plan (batch.cpp): per radius group (0: r 0..4,
// 1: unused, radii above PF_BATCH_R_MAX are rejected) the image descriptors and the flat wave-tile list, the variant
// of each image, and the variant set each group uses.
struct PlanTables {
    std::vector<BatchImg> imgs[2];
    std::vector<BatchTask> tasks[2];
    std::vector<int32_t> variant;
    int used[2] = {0, 0};
};
pf_status build_plan_tables(int32_t n, const int32_t *h, const int32_t *w, const int32_t *r, const int32_t *kind,
                            const int64_t *pix_off, const int64_t *filt_off, int64_t npix, int64_t nfilt,
                            int32_t flags, PlanTables *t);
int64_t check_plan_tables(const PlanTables &t, int64_t npix, std::string *first);

// Workgroups of a batch launch over `ntiles` wave tiles: `blocks_per_cu`
// per compute unit (from the tune table), at most what fits at once, at
// most one tile per wave.
int batch_grid(int group, bool exact, int mask, int wpg, int64_t ntiles);

// Size class used by the tune table.
inline int size_class(int64_t pixels) {
    return pixels < 256 * 256 ? 0 : (pixels > 1024 * 1024 ? 2 : 1);
}

// Device properties the launchers need (cached per device).
struct DevInfo {
    int device = -1;
    int cus = 0;
    std::string arch;
};
const DevInfo &dev_info();

// Thread-local error text.
pf_status fail(pf_status s, const std::string &msg);
pf_status fail_hip(hipError_t e, const char *what);
void clear_error();

// Launchers (kernels.hip). All validate nothing: callers have already.
// fa: 2D taps (PF_VAR_DIRECT) or fx; fb: fy (ignored for PF_VAR_DIRECT).
hipError_t launch_f32(int r, int var, bool exact, const float *in, const float *fa, const float *fb, float *out,
                      int h, int w, int by, int wpg, hipStream_t s);
// var: PF_VAR_DIRECT (v_dot4) or PF_VAR_MFMA (int8 matrix cores, u8_mfma.hip).
hipError_t launch_u8(int r, int var, const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h,
                     int w, int shift, int by, int wpg, hipStream_t s);
hipError_t launch_u8_mfma(int r, const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h, int w,
                          int shift, int rpw, int wpg, hipStream_t s);
// Whether the uint8 variant runs at radius r with this launch shape.
bool u8_variant_ok(int var, int r, int by, int wpg);
// Persistent batch kernel over images with r <= 4 (group 0; group 1 is not
// built and fails with hipErrorInvalidValue), compiled with the variants of
// `mask` (see batch_mask).
hipError_t launch_batch(int group, bool exact, int mask, const BatchImg *imgs, const BatchTask *tasks,
                        int ntasks, int grid, int wpg, const float *in, const float *filt, float *out,
                        hipStream_t s);
// Fused chain of `passes` 2D passes under a border rule (chain.hip); also
// the single-pass filter for borders other than clamp.
hipError_t launch_chain(int r, bool exact, const float *in, const float *filt, float *out, int h, int w, int passes,
                        int border, hipStream_t s);
// Reductions (reduce.hip): workspace sizes and the two-launch sum and
// histogram.
size_t sum_workspace_bytes(int64_t n);
size_t hist_workspace_bytes(int64_t n);
hipError_t launch_sum(const float *x, int64_t n, double *out, void *workspace, hipStream_t s);
hipError_t launch_hist(const uint8_t *x, int64_t n, int64_t *hist, void *workspace, hipStream_t s);
// Reduction requests of a server batch (reduce.hip). in / out are absolute
// device addresses (the input array; double[2] or int64_t[256] result);
// `first` is the request's first slot in the batch workspace: chunk
// partials (double) for sums, span sub-histograms (256 x uint32) for
// histograms; `op` is PF_OP_SUM_F32 or PF_OP_HIST_U8.
struct ReduceReq {
    int64_t in, n, out, first;
    int32_t op, pad;
};
// Part `part` (chunk or span) of request `req`.
struct ReduceTask {
    int32_t req, part;
};
// Chunks (sum) or spans (histogram) of an n-element request.
int64_t reduce_parts(int op, int64_t n);
// All sums, then all histograms of a batch: two launches each.
hipError_t launch_reduce_batch(const ReduceReq *reqs, const int32_t *sum_ids, int nsum, const ReduceTask *sum_tasks,
                               int n_sum_tasks, const int32_t *hist_ids, int nhist, const ReduceTask *hist_tasks,
                               int n_hist_tasks, double *partial, uint32_t *sub, hipStream_t s);
// The sum's static device scratch (reduce.hip): its capacity in elements and
// its address on the current device.
int64_t sum_noalloc_max();
hipError_t sum_scratch(void **ptr);
// Workgroups of the batch kernel that fit on the device at once.
int batch_grid_limit(int group, bool exact, int mask, int wpg);
void *batch_kernel_fn(int group, bool exact, int mask);

// Per-radius FP32 launchers, each defined in its own instantiation unit.
template <int R>
hipError_t launch_f32_radius(int var, bool exact, const float *in, const float *fa, const float *fb, float *out,
                             int h, int w, int by, int wpg, hipStream_t s);
#define PF_DECL_RADIUS(R)                                                                                  \
    template <>                                                                                            \
    hipError_t launch_f32_radius<R>(int var, bool exact, const float *in, const float *fa, const float *fb, \
                                    float *out, int h, int w, int by, int wpg, hipStream_t s);
PF_DECL_RADIUS(0)
PF_DECL_RADIUS(1)
PF_DECL_RADIUS(2)
PF_DECL_RADIUS(3)
PF_DECL_RADIUS(4)
PF_DECL_RADIUS(5)
PF_DECL_RADIUS(6)
PF_DECL_RADIUS(7)
PF_DECL_RADIUS(8)
#undef PF_DECL_RADIUS

// Batch kernels per (radius group, exact, variant mask), each in its own
// unit. Masks: bit v for variant v: 1 (direct only), 2 (separable only)
// and 3 (both). Only group 0 (radii 0..PF_BATCH_R_MAX) is built. The separable-as-2D
// variant is not compiled into batch kernels (it runs in single-image calls
// only) so that the persistent kernel stays small.
template <int G, int E, int M>
void *batch_fn();
template <int G, int E, int M>
hipError_t launch_batch_g(const BatchImg *imgs, const BatchTask *tasks, int ntasks, int grid, int wpg,
                          const float *in, const float *filt, float *out, hipStream_t s);
#define PF_DECL_BATCH(G, E, M)                                                                                 \
    template <>                                                                                                \
    void *batch_fn<G, E, M>();                                                                                 \
    template <>                                                                                                \
    hipError_t launch_batch_g<G, E, M>(const BatchImg *imgs, const BatchTask *tasks, int ntasks, int grid,      \
                                       int wpg, const float *in, const float *filt, float *out, hipStream_t s);
PF_DECL_BATCH(0, 0, 1)
PF_DECL_BATCH(0, 1, 1)
PF_DECL_BATCH(0, 0, 2)
PF_DECL_BATCH(0, 1, 2)
PF_DECL_BATCH(0, 0, 3)
PF_DECL_BATCH(0, 1, 3)
#undef PF_DECL_BATCH

// Smallest compiled variant mask of a group that covers `used` (bit v set
// if some image runs variant v).
inline int batch_mask(int group, int used) {
    if (group == 1) return 3;
    if ((used & ~1) == 0) return 1;
    if ((used & ~2) == 0) return 2;
    return 3;
}

// Tune table lookups (tune.cpp): single-image calls, and the persistent
// batch kernel of plans and servers.
pf_tune_entry tune_lookup(int kind, int r, int64_t pixels);
pf_tune_entry tune_lookup_batch(int kind, int r, int64_t pixels);
// Workgroups per compute unit of persistent batch launches (tune.cpp).
int tune_batch_blocks_per_cu();

bool valid_shape(int by, int wpg);

}  // namespace pf
