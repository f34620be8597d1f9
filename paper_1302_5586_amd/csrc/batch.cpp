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
    // Two groups: radii 0..4 (index 0) and 5..8 (index 1).
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

    pf_batch_plan *p = new (std::nothrow) pf_batch_plan;
    if (!p) return fail(PF_ENOMEM, "plan allocation");
    p->n = n;
    p->npix = npix;
    p->nfilt = nfilt;
    p->flags = flags;
    (void)hipGetDevice(&p->device);
    p->variant.resize(n);

    std::vector<BatchImg> imgs[2];
    int64_t ntiles[2] = {0, 0};
    int used[2] = {0, 0};
    for (int i = 0; i < n; ++i) {
        const int64_t px = (int64_t)h[i] * w[i];
        pf_tune_entry e;
        if (flags & PF_BATCH_NO_TUNE) {
            e.variant = kind[i] == PF_KIND_SEP ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
            e.rows_per_wave = 16;
        } else {
            e = tune_lookup(kind[i], r[i], px);
        }
        int var = kind[i] == PF_KIND_2D ? PF_VAR_DIRECT : (e.variant == PF_VAR_SEP_DIRECT ? PF_VAR_SEP_DIRECT : PF_VAR_SEPARABLE);
        p->variant[i] = var;
        const int g = r[i] <= 4 ? 0 : 1;
        used[g] |= 1 << var;
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
        if (ntiles[g] + nt > INT32_MAX) {
            delete p;
            return fail(PF_EUNSUPPORTED, "batch has more than 2^31-1 wave tiles");
        }
        ntiles[g] += nt;
        imgs[g].push_back(d);
    }
    std::vector<BatchTask> tasks[2];
    size_t bytes = 0;
    size_t off_imgs[2], off_tasks[2];
    for (int g = 0; g < 2; ++g) {
        p->ntasks[g] = ntiles[g];
        p->mask[g] = batch_mask(g, used[g]);
        p->grid[g] = ntiles[g] ? batch_grid(g, (flags & PF_FLAG_EXACT) != 0, p->mask[g], p->wpg, ntiles[g]) : 0;
        tasks[g].reserve((size_t)ntiles[g]);
        for (size_t i = 0; i < imgs[g].size(); ++i) append_tiles(tasks[g], (int32_t)i, imgs[g][i]);
        off_imgs[g] = bytes;
        bytes += imgs[g].size() * sizeof(BatchImg);
        bytes = (bytes + 255) & ~(size_t)255;
        off_tasks[g] = bytes;
        bytes += tasks[g].size() * sizeof(BatchTask);
        bytes = (bytes + 255) & ~(size_t)255;
    }
    hipError_t e = hipMalloc(&p->dev, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "plan descriptor allocation");
    }
    std::vector<char> host(std::max<size_t>(bytes, 256), 0);
    for (int g = 0; g < 2; ++g) {
        if (!imgs[g].empty()) memcpy(host.data() + off_imgs[g], imgs[g].data(), imgs[g].size() * sizeof(BatchImg));
        if (!tasks[g].empty()) memcpy(host.data() + off_tasks[g], tasks[g].data(), tasks[g].size() * sizeof(BatchTask));
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
