// Batch plans: many images of uneven sizes and radii in one persistent
// launch, optionally replayed from a hipGraph.
//
// The batch is described the way the paper rewrites OP2's kernel for
// PENCIL (Sec. III-A): no arrays of pointers, only arenas plus per-image
// offsets. Every image's outputs are independent iterations (Sec. II-B.3),
// so all images' wave tiles form one flat list that a fixed grid of
// workgroups walks with a static stride.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "pf_internal.h"

struct pf_batch_plan {
    int32_t n = 0;
    int64_t npix = 0, nfilt = 0;
    int32_t flags = 0;
    int device = -1;
    std::vector<int32_t> variant;  // per image
    // Radius groups: 0 (radii 0..PF_BATCH_R_MAX); index 1 is kept empty.
    int64_t ntasks[2] = {0, 0};
    int32_t grid[2] = {0, 0};
    int32_t mask[2] = {3, 3};  // compiled variant set of each group's kernel
    int32_t wpg = 4;
    void *dev = nullptr;  // descriptors and tile lists, one allocation
    const pf::BatchImg *imgs[2] = {nullptr, nullptr};
    const pf::BatchTask *tasks[2] = {nullptr, nullptr};
    // Graph replay state.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node[2] = {nullptr, nullptr};
    const float *g_in = nullptr, *g_filt = nullptr;
    float *g_out = nullptr;
    std::mutex mu;
};

namespace pf {

// Sets kernel parameters for group g of plan p (pointers must outlive use).
struct BatchArgs {
    const BatchImg *imgs;
    const BatchTask *tasks;
    int ntasks;
    const float *in;
    const float *filt;
    float *out;
    void *params[6];
    void fill() {
        params[0] = &imgs;
        params[1] = &tasks;
        params[2] = &ntasks;
        params[3] = &in;
        params[4] = &filt;
        params[5] = &out;
    }
};

static hipKernelNodeParams node_params(pf_batch_plan *p, int g, BatchArgs &a) {
    a.fill();
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    kp.func = batch_kernel_fn(g, (p->flags & PF_FLAG_EXACT) != 0, p->mask[g]);
    kp.gridDim = dim3(p->grid[g]);
    kp.blockDim = dim3(p->wpg * 64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = a.params;
    kp.extra = nullptr;
    return kp;
}

// Validates a batch description (sizes, radii, kinds, arena ranges, no two
// images overlapping) and builds the plan's host tables: per radius group
// (all radii are in group 0, 0..PF_BATCH_R_MAX) the image descriptors with their variant and tile height from
// the batch context of the tune table, and the flat list of wave tiles.
pf_status build_plan_tables(int32_t n, const int32_t *h, const int32_t *w, const int32_t *r, const int32_t *kind,
                            const int64_t *pix_off, const int64_t *filt_off, int64_t npix, int64_t nfilt,
                            int32_t flags, PlanTables *t) {
    if (n < 1) return fail(PF_EINVAL, "batch needs at least one image");
    if (!h || !w || !r || !kind || !pix_off || !filt_off) return fail(PF_EINVAL, "null descriptor array");
    if (npix < 1 || nfilt < 1) return fail(PF_EINVAL, "arena sizes must be >= 1");
    if (flags & ~(PF_FLAG_EXACT | PF_BATCH_GRAPH | PF_BATCH_NO_TUNE)) return fail(PF_EINVAL, "unknown flags");

    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve(n);
    for (int i = 0; i < n; ++i) {
        const std::string at = " (image " + std::to_string(i) + ")";
        if (h[i] < 1 || w[i] < 1) return fail(PF_EINVAL, "image sizes must be >= 1" + at);
        if (r[i] < 0 || r[i] > PF_R_MAX) return fail(PF_EINVAL, "radius outside 0.." + std::to_string(PF_R_MAX) + at);
        if (r[i] > PF_BATCH_R_MAX)
            return fail(PF_EUNSUPPORTED,
                        "batches take radii 0.." + std::to_string(PF_BATCH_R_MAX) + " (larger: single-image calls)" + at);
        if (kind[i] != PF_KIND_2D && kind[i] != PF_KIND_SEP) return fail(PF_EINVAL, "unknown filter kind" + at);
        const int64_t px = (int64_t)h[i] * w[i];
        const int64_t k = 2 * r[i] + 1;
        const int64_t nf = kind[i] == PF_KIND_2D ? k * k : 2 * k;
        if (pix_off[i] < 0 || pix_off[i] > npix - px) return fail(PF_EINVAL, "image outside the pixel arena" + at);
        if (filt_off[i] < 0 || filt_off[i] > nfilt - nf) return fail(PF_EINVAL, "filter outside the filter arena" + at);
        spans.push_back({pix_off[i], px});
    }
    // Outputs of distinct images must not overlap (restrict, Sec. II-B.1).
    std::sort(spans.begin(), spans.end());
    for (int i = 1; i < n; ++i)
        if (spans[i - 1].first + spans[i - 1].second > spans[i].first)
            return fail(PF_EALIAS, "two images overlap in the pixel arena");

    t->variant.resize(n);
    int64_t ntiles[2] = {0, 0};
    for (int i = 0; i < n; ++i) {
        const int64_t px = (int64_t)h[i] * w[i];
        pf_tune_entry e;
        if (flags & PF_BATCH_NO_TUNE) {
            e.variant = kind[i] == PF_KIND_SEP ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
            e.rows_per_wave = 16;
        } else {
            e = tune_lookup_batch(kind[i], r[i], px);
        }
        const int var = kind[i] == PF_KIND_2D ? PF_VAR_DIRECT : PF_VAR_SEPARABLE;
        t->variant[i] = var;
        const int g = r[i] <= 4 ? 0 : 1;
        t->used[g] |= 1 << var;
        BatchImg d;
        d.in_off = pix_off[i];
        d.out_off = pix_off[i];
        d.filt_off = filt_off[i];
        d.h = h[i];
        d.w = w[i];
        d.r = r[i];
        d.var = var;
        d.by = e.rows_per_wave;
        const int64_t nt = set_strips(d);
        if (ntiles[g] + nt > INT32_MAX) return fail(PF_EUNSUPPORTED, "batch has more than 2^31-1 wave tiles");
        ntiles[g] += nt;
        t->imgs[g].push_back(d);
    }
    for (int g = 0; g < 2; ++g) {
        t->tasks[g].reserve((size_t)ntiles[g]);
        for (size_t i = 0; i < t->imgs[g].size(); ++i) append_tiles(t->tasks[g], (int32_t)i, t->imgs[g][i]);
    }
    return PF_OK;
}

// Replays, on the host, where every wave tile of the tables reads and
// writes, with the geometry functions the FP32 strip kernel itself calls
// (strip_mode, lane_col, vec_load_col, halo_load_col, tile_strip): each
// tile must name a valid image and a strip and row band inside it; each
// 16-byte load of a lane (kStripFast, kStripEdge), each halo load of an
// aligned strip (kStripFast) and each plain 16-byte store (kStripFast
// without halo lanes) must lie in [0, w) of its row; and the image must lie
// inside the pixel arena. Loads of single clamped columns and stores
// through range-checked buffer resources stay in bounds by construction.
// Returns the number of violations; the first is described in *first.
int64_t check_plan_tables(const PlanTables &t, int64_t npix, std::string *first) {
    int64_t bad = 0;
    auto report = [&](int g, size_t k, const std::string &what) {
        if (!bad++) *first = "group " + std::to_string(g) + " tile " + std::to_string(k) + ": " + what;
    };
    for (int g = 0; g < 2; ++g) {
        const std::vector<BatchImg> &imgs = t.imgs[g];
        for (const BatchImg &d : imgs)
            if (d.in_off < 0 || d.in_off + (int64_t)d.h * d.w > npix || d.out_off < 0 ||
                d.out_off + (int64_t)d.h * d.w > npix) {
                report(g, 0, "image outside the arena");
            }
        for (size_t k = 0; k < t.tasks[g].size(); ++k) {
            const BatchTask tk = t.tasks[g][k];
            if (tk.img < 0 || tk.img >= (int)imgs.size()) {
                report(g, k, "image index out of range");
                continue;
            }
            const BatchImg &d = imgs[tk.img];
            if (tk.tile < 0 || tk.tile >= d.strips_x * d.strips_y) {
                report(g, k, "tile number out of range");
                continue;
            }
            int sx = 0, sy = 0;
            tile_strip(kTileColMajorF32, tk.tile, d.strips_x, d.strips_y, sx, sy);
            const int x0 = sx * strip_width(d.r), y0 = sy * d.by;
            const int rows = std::min(d.by, d.h - y0);
            if (x0 < 0 || x0 >= d.w || y0 < 0 || rows < 1 || y0 + rows > d.h) {
                report(g, k, "strip origin or row band outside the image");
                continue;
            }
            const int mode = strip_mode(d.r, x0, d.w);
            for (int lane = 0; lane < 64; ++lane) {
                const int xs = lane_col(d.r, x0, lane);
                if (mode != kStripTiny) {
                    const int c = vec_load_col(d.r, mode, xs, d.w);
                    if (c < 0 || c + 4 > d.w) report(g, k, "16-byte load outside the row (lane " + std::to_string(lane) + ")");
                }
                if (mode == kStripFast && aligned_strip(d.r)) {
                    const int c = halo_load_col(d.r, lane < 32, x0, d.w);
                    if (c < 0 || c + d.r > d.w) report(g, k, "halo load outside the row (lane " + std::to_string(lane) + ")");
                }
                if (mode == kStripFast && idle_lanes(d.r) == 0 && (xs < 0 || xs + 4 > d.w))
                    report(g, k, "16-byte store outside the row (lane " + std::to_string(lane) + ")");
            }
        }
    }
    return bad;
}

}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_batch_plan_create(int32_t n, const int32_t *__restrict h, const int32_t *__restrict w,
                               const int32_t *__restrict r, const int32_t *__restrict kind,
                               const int64_t *__restrict pix_off, const int64_t *__restrict filt_off, int64_t npix,
                               int64_t nfilt, int32_t flags, pf_batch_plan **const __restrict plan) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "null plan out-parameter");
    *plan = nullptr;
    PlanTables t;
    pf_status st = build_plan_tables(n, h, w, r, kind, pix_off, filt_off, npix, nfilt, flags, &t);
    if (st) return st;

    pf_batch_plan *p = new (std::nothrow) pf_batch_plan;
    if (!p) return fail(PF_ENOMEM, "plan allocation");
    p->n = n;
    p->npix = npix;
    p->nfilt = nfilt;
    p->flags = flags;
    (void)hipGetDevice(&p->device);
    p->variant = t.variant;
    size_t bytes = 0;
    size_t off_imgs[2], off_tasks[2];
    for (int g = 0; g < 2; ++g) {
        const int64_t ntiles = (int64_t)t.tasks[g].size();
        p->ntasks[g] = ntiles;
        p->mask[g] = batch_mask(g, t.used[g]);
        p->grid[g] = ntiles ? batch_grid(g, (flags & PF_FLAG_EXACT) != 0, p->mask[g], p->wpg, ntiles) : 0;
        off_imgs[g] = bytes;
        bytes += t.imgs[g].size() * sizeof(BatchImg);
        bytes = (bytes + 255) & ~(size_t)255;
        off_tasks[g] = bytes;
        bytes += t.tasks[g].size() * sizeof(BatchTask);
        bytes = (bytes + 255) & ~(size_t)255;
    }
    hipError_t e = hipMalloc(&p->dev, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "plan descriptor allocation");
    }
    std::vector<char> host(std::max<size_t>(bytes, 256), 0);
    for (int g = 0; g < 2; ++g) {
        if (!t.imgs[g].empty()) memcpy(host.data() + off_imgs[g], t.imgs[g].data(), t.imgs[g].size() * sizeof(BatchImg));
        if (!t.tasks[g].empty())
            memcpy(host.data() + off_tasks[g], t.tasks[g].data(), t.tasks[g].size() * sizeof(BatchTask));
        p->imgs[g] = (const BatchImg *)((char *)p->dev + off_imgs[g]);
        p->tasks[g] = (const BatchTask *)((char *)p->dev + off_tasks[g]);
    }
    e = hipMemcpy(p->dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        delete p;
        return fail_hip(e, "plan descriptor upload");
    }
    *plan = p;
    return PF_OK;
}

pf_status pf_batch_plan_check(int32_t n, const int32_t *__restrict h, const int32_t *__restrict w,
                              const int32_t *__restrict r, const int32_t *__restrict kind,
                              const int64_t *__restrict pix_off, const int64_t *__restrict filt_off, int64_t npix,
                              int64_t nfilt, int32_t flags, int64_t *const __restrict tiles,
                              int64_t *const __restrict violations) {
    clear_error();
    if (!tiles || !violations) return fail(PF_EINVAL, "null out-parameter");
    *tiles = *violations = 0;
    PlanTables t;
    pf_status st = build_plan_tables(n, h, w, r, kind, pix_off, filt_off, npix, nfilt, flags, &t);
    if (st) return st;
    std::string first;
    *tiles = (int64_t)(t.tasks[0].size() + t.tasks[1].size());
    *violations = check_plan_tables(t, npix, &first);
    if (*violations) return fail(PF_EINVAL, first);
    return PF_OK;
}

pf_status pf_batch_plan_run(pf_batch_plan *p, int64_t npix, int64_t nfilt, const float *__restrict in,
                            const float *__restrict filt, float *__restrict out, void *stream) {
    clear_error();
    if (!p) return fail(PF_EINVAL, "null plan");
    if (npix != p->npix || nfilt != p->nfilt) return fail(PF_EINVAL, "arena sizes differ from the plan's");
    if (!in || !filt || !out) return fail(PF_EINVAL, "null arena pointer");
    if (((uintptr_t)in | (uintptr_t)filt | (uintptr_t)out) % 4) return fail(PF_EINVAL, "arenas must be 4-byte aligned");
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out, nb = (uintptr_t)npix * 4;
    if (a < b + nb && b < a + nb) return fail(PF_EALIAS, "input and output arenas overlap (restrict)");
    const uintptr_t f = (uintptr_t)filt, fb = (uintptr_t)nfilt * 4;
    if (f < b + nb && b < f + fb) return fail(PF_EALIAS, "filter and output arenas overlap (restrict)");
    hipStream_t s = (hipStream_t)stream;
    const bool exact = (p->flags & PF_FLAG_EXACT) != 0;
    std::lock_guard<std::mutex> lk(p->mu);
    if (!(p->flags & PF_BATCH_GRAPH)) {
        for (int g = 0; g < 2; ++g) {
            if (!p->ntasks[g]) continue;
            hipError_t e = launch_batch(g, exact, p->mask[g], p->imgs[g], p->tasks[g], (int)p->ntasks[g], p->grid[g],
                                        p->wpg, in, filt, out, s);
            if (e != hipSuccess) return fail_hip(e, "batch launch");
        }
        return PF_OK;
    }
    hipError_t e = hipSuccess;
    if (!p->exec) {
        // Build the graph once: one kernel node per non-empty group, in order.
        if ((e = hipGraphCreate(&p->graph, 0)) != hipSuccess) return fail_hip(e, "graph create");
        hipGraphNode_t prev = nullptr;
        for (int g = 0; g < 2; ++g) {
            if (!p->ntasks[g]) continue;
            BatchArgs a{p->imgs[g], p->tasks[g], (int)p->ntasks[g], in, filt, out, {}};
            hipKernelNodeParams kp = node_params(p, g, a);
            e = hipGraphAddKernelNode(&p->node[g], p->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
            if (e != hipSuccess) return fail_hip(e, "graph kernel node");
            prev = p->node[g];
        }
        if ((e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess) {
            p->exec = nullptr;
            return fail_hip(e, "graph instantiate");
        }
        p->g_in = in;
        p->g_filt = filt;
        p->g_out = out;
    } else if (in != p->g_in || filt != p->g_filt || out != p->g_out) {
        // Re-point the replay at the new arenas.
        for (int g = 0; g < 2; ++g) {
            if (!p->ntasks[g]) continue;
            BatchArgs a{p->imgs[g], p->tasks[g], (int)p->ntasks[g], in, filt, out, {}};
            hipKernelNodeParams kp = node_params(p, g, a);
            if ((e = hipGraphExecKernelNodeSetParams(p->exec, p->node[g], &kp)) != hipSuccess)
                return fail_hip(e, "graph node update");
        }
        p->g_in = in;
        p->g_filt = filt;
        p->g_out = out;
    }
    if ((e = hipGraphLaunch(p->exec, s)) != hipSuccess) return fail_hip(e, "graph launch");
    return PF_OK;
}

pf_status pf_batch_plan_variants(const pf_batch_plan *p, int32_t n, int32_t *__restrict variant) {
    clear_error();
    if (!p || !variant) return fail(PF_EINVAL, "null argument");
    if (n != p->n) return fail(PF_EINVAL, "n differs from the plan's image count");
    for (int i = 0; i < n; ++i) variant[i] = p->variant[i];
    return PF_OK;
}

pf_status pf_batch_plan_info(const pf_batch_plan *p, int64_t *const __restrict tasks, int32_t *const __restrict launches,
                             int32_t *const __restrict grid) {
    clear_error();
    if (!p || !tasks || !launches || !grid) return fail(PF_EINVAL, "null argument");
    *tasks = p->ntasks[0] + p->ntasks[1];
    *launches = (p->ntasks[0] > 0) + (p->ntasks[1] > 0);
    *grid = p->ntasks[0] ? p->grid[0] : p->grid[1];
    return PF_OK;
}

pf_status pf_batch_plan_destroy(pf_batch_plan *p) {
    clear_error();
    if (!p) return PF_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
    return PF_OK;
}

}  // extern "C"
