// Tune table and autotuner: profile-based tuning of the launch shape and of
// the variant a separable filter runs as (the paper's compilation flow ends
// in "profile-based iterative compilation and auto-tuning", Sec. II, Fig. 1).
//
// The table is keyed by (context, kind, radius, size class). Context 0
// holds the shapes of single-image calls, context 1 those of the persistent
// batch kernel (batch plans and servers): the two launch differently (one
// image and many small waves against a fixed grid walking many images), so
// they are tuned and stored apart and neither tuner touches the other's
// entries. Results never depend on the launch shape (each output's
// arithmetic is fixed), only on the variant, and the variant depends only
// on the key.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "pf_internal.h"

namespace pf {

namespace {

// Tile heights (multiples of 4 in 8..64) whose rows fill whole chunks of
// the FP32 strip's row pipeline for radius r (no one-by-one tail rows).
std::vector<int> whole_chunk_heights(int r, int chunk) {
    const int ch = chunk_rows_of(r, chunk);
    std::vector<int> v;
    for (int by = ch; by <= 64; by += ch)
        if (by % 4 == 0 && by >= 8) v.push_back(by);
    return v;
}


constexpr int kKinds = 3;  // PF_KIND_2D, PF_KIND_SEP, PF_KIND_U8
constexpr int kSizes = 3;
constexpr int kContexts = 2;  // PF_TUNE_SINGLE, PF_TUNE_BATCH
constexpr int kBatchWaves = 4;  // waves per workgroup of persistent batch launches

// Workgroups per compute unit of a persistent batch launch. One (four
// waves, one per SIMD) measured best on MI355X: the fewest tiles in flight
// keep the window of HBM pages the batch touches at once compact.
constexpr int kBatchBlocksPerCu = 1;
constexpr int kBatchBlocksPerCuMax = 8;

struct Table {
    pf_tune_entry e[kContexts][kKinds][PF_R_MAX + 1][kSizes];
    int batch_blocks_per_cu = kBatchBlocksPerCu;
};

pf_tune_entry default_entry(int ctx, int kind, int r, int sc) {
    pf_tune_entry e;
    e.kind = kind;
    e.r = r;
    e.size_class = sc;
    e.context = ctx;
    e.variant = (kind == PF_KIND_SEP) ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
    // Defaults measured on MI355X: 16-row tiles for small images, for
    // batches and for the uint8 path, 32-row tiles otherwise. uint8 at radii
    // the matrix-core kernel runs (1.5x faster than v_dot4 at 1080p RGB,
    // 7 x 7): that kernel, four waves of 16 rows per workgroup.
    const bool u8_mfma = kind == PF_KIND_U8 && ctx == PF_TUNE_SINGLE && r >= 1 && r <= PF_U8_MFMA_R_MAX;
    if (u8_mfma) e.variant = PF_VAR_MFMA;
    e.rows_per_wave = (ctx == PF_TUNE_BATCH || sc == 0 || kind == PF_KIND_U8) ? 16 : 32;
    e.waves_per_group = ctx == PF_TUNE_BATCH ? kBatchWaves : (kind == PF_KIND_U8 && !u8_mfma ? 1 : 4);
    e.us = 0.0f;
    return e;
}

Table make_default() {
    Table t;
    for (int c = 0; c < kContexts; ++c)
        for (int k = 0; k < kKinds; ++k)
            for (int r = 0; r <= PF_R_MAX; ++r)
                for (int s = 0; s < kSizes; ++s) t.e[c][k][r][s] = default_entry(c, k, r, s);
    return t;
}

std::mutex g_mu;
Table g_table = make_default();

bool entry_ok(const pf_tune_entry &e) {
    if (e.context < 0 || e.context >= kContexts) return false;
    if (e.kind < 0 || e.kind >= kKinds || e.r < 0 || e.r > PF_R_MAX || e.size_class < 0 || e.size_class >= kSizes)
        return false;
    if (!valid_shape(e.rows_per_wave, e.waves_per_group)) return false;
    if (e.context == PF_TUNE_BATCH) {
        // Batches hold FP32 images only; their kernel runs four waves per
        // workgroup and compiles only the direct and separable bodies.
        if (e.kind == PF_KIND_U8 || e.waves_per_group != kBatchWaves) return false;
        return e.variant == (e.kind == PF_KIND_SEP ? PF_VAR_SEPARABLE : PF_VAR_DIRECT);
    }
    // A separable filter called alone may also run as 2D taps fy[i] * fx[j].
    if (e.kind == PF_KIND_SEP)
        return e.variant == PF_VAR_SEPARABLE || (e.variant == PF_VAR_SEP_DIRECT && e.r <= PF_SEP_DIRECT_R_MAX);
    // uint8 may run on v_dot4 or on the int8 matrix cores.
    if (e.kind == PF_KIND_U8) return u8_variant_ok(e.variant, e.r, e.rows_per_wave, e.waves_per_group);
    return e.variant == PF_VAR_DIRECT;
}

// Minimal reader for the table's own JSON: numbers keyed by the field
// names inside each object of the "entries" array.
bool parse_number(const std::string &obj, const char *key, double *out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char *end = nullptr;
    const double v = strtod(obj.c_str() + p + 1, &end);
    if (end == obj.c_str() + p + 1) return false;
    *out = v;
    return true;
}

}  // namespace

pf_tune_entry tune_lookup(int kind, int r, int64_t pixels) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table.e[PF_TUNE_SINGLE][kind][r][size_class(pixels)];
}

pf_tune_entry tune_lookup_batch(int kind, int r, int64_t pixels) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table.e[PF_TUNE_BATCH][kind][r][size_class(pixels)];
}

int tune_batch_blocks_per_cu() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_table.batch_blocks_per_cu;
}

// ---------------------------------------------------------------- autotune

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Median time (us) of one launch, from `trials` groups of `reps` launches
// that rotate over `nbuf` disjoint buffer sets.
template <class F>
pf_status time_launch(F &&launch, int nbuf, int reps, int trials, hipStream_t s, float *us) {
    Timer t;
    std::vector<float> v;
    for (int w = 0; w < 3; ++w) {
        hipError_t e = launch(w % nbuf);
        if (e != hipSuccess) return fail_hip(e, "autotune launch");
    }
    for (int tr = 0; tr < trials; ++tr) {
        (void)hipEventRecord(t.a, s);
        for (int i = 0; i < reps; ++i) {
            hipError_t e = launch(i % nbuf);
            if (e != hipSuccess) return fail_hip(e, "autotune launch");
        }
        (void)hipEventRecord(t.b, s);
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return fail_hip(e, "autotune sync");
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t.a, t.b);
        v.push_back(ms * 1000.0f / reps);
    }
    std::sort(v.begin(), v.end());
    *us = v[v.size() / 2];
    return PF_OK;
}

// Representative image of each size class, and how many of them one timed
// batch launch holds (context 1 entries are timed on such a batch, context
// 0 entries on single launches of one image).
void class_shape(int sc, int kind, int *h, int *w, int *n) {
    static const int hs[kSizes] = {160, 600, 4096};
    static const int ws[kSizes] = {200, 700, 4096};
    static const int ns[kSizes] = {1024, 96, 4};
    *h = hs[sc];
    *w = ws[sc];
    *n = ns[sc];
    if (kind == PF_KIND_U8 && sc == 2) {  // planar RGB at 1080p
        *h = 1080;
        *w = 1920;
    }
}

// Time one persistent batch launch over n images of h x w with radius r,
// filter kind `kind` and row tiles of `by`, reading in[] and writing out[]
// (n*h*w floats each) with the weights at filt.
pf_status time_batch_class(int kind, int r, int h, int w, int n, int by, const float *in, float *out,
                           const float *filt, int reps, hipStream_t s, float *us) {
    const int g = r <= 4 ? 0 : 1;
    const int var = kind == PF_KIND_SEP ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
    const int mask = batch_mask(g, 1 << var);
    std::vector<BatchImg> imgs(n);
    int64_t ntiles = 0;
    for (int i = 0; i < n; ++i) {
        BatchImg &d = imgs[i];
        d.in_off = d.out_off = (int64_t)i * h * w;
        d.filt_off = 0;
        d.h = h;
        d.w = w;
        d.r = r;
        d.var = var;
        d.by = by;
        ntiles += set_strips(d);
    }
    const int wpg = 4;
    const int grid = batch_grid(g, false, mask, wpg, ntiles);
    std::vector<BatchTask> tasks;
    for (int i = 0; i < n; ++i) append_tiles(tasks, i, imgs[i]);
    void *dev = nullptr;
    const size_t bi = imgs.size() * sizeof(BatchImg), bt = tasks.size() * sizeof(BatchTask);
    hipError_t e = hipMalloc(&dev, bi + bt);
    if (e != hipSuccess) return fail_hip(e, "autotune descriptors");
    e = hipMemcpy(dev, imgs.data(), bi, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((char *)dev + bi, tasks.data(), bt, hipMemcpyHostToDevice);
    pf_status st = PF_OK;
    if (e != hipSuccess) {
        st = fail_hip(e, "autotune descriptors");
    } else {
        st = time_launch(
            [&](int) {
                return launch_batch(g, false, mask, (const BatchImg *)dev, (const BatchTask *)((char *)dev + bi),
                                    (int)tasks.size(), grid, wpg, in, filt, out, s);
            },
            1, reps, 5, s, us);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(dev);
    return st;
}

}  // namespace

}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_tune_lookup(int32_t kind, int32_t r, int64_t pixels, int32_t context, pf_tune_entry *const __restrict e) {
    clear_error();
    if (!e) return fail(PF_EINVAL, "null output");
    if (kind < 0 || kind >= kKinds || r < 0 || r > PF_R_MAX || pixels < 1) return fail(PF_EINVAL, "bad tune key");
    if (context != PF_TUNE_SINGLE && !(context == PF_TUNE_BATCH && kind != PF_KIND_U8))
        return fail(PF_EINVAL, "bad tune context");
    std::lock_guard<std::mutex> lk(g_mu);
    *e = g_table.e[context][kind][r][size_class(pixels)];
    return PF_OK;
}

pf_status pf_tune_set(int32_t n, const pf_tune_entry *__restrict entries) {
    clear_error();
    if (n < 0 || (n > 0 && !entries)) return fail(PF_EINVAL, "bad entry list");
    for (int i = 0; i < n; ++i)
        if (!entry_ok(entries[i])) return fail(PF_EINVAL, "invalid tune entry " + std::to_string(i));
    Table t = make_default();
    for (int i = 0; i < n; ++i) {
        const pf_tune_entry &e = entries[i];
        t.e[e.context][e.kind][e.r][e.size_class] = e;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_table = t;
    return PF_OK;
}

pf_status pf_tune_reset(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    g_table = make_default();
    return PF_OK;
}

pf_status pf_tune_save(const char *path) {
    clear_error();
    if (!path) return fail(PF_EINVAL, "null path");
    Table t;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        t = g_table;
    }
    FILE *f = fopen(path, "w");
    if (!f) return fail(PF_EINVAL, std::string("cannot write ") + path);
    const DevInfo &d = dev_info();
    fprintf(f, "{\n  \"library\": \"%s\",\n  \"device_arch\": \"%s\",\n  \"batch_blocks_per_cu\": %d,\n  \"entries\": [\n",
            pf_version(), d.arch.c_str(), t.batch_blocks_per_cu);
    bool first = true;
    for (int c = 0; c < kContexts; ++c)
        for (int k = 0; k < kKinds; ++k) {
            if (c == PF_TUNE_BATCH && k == PF_KIND_U8) continue;
            for (int r = 0; r <= PF_R_MAX; ++r)
                for (int s = 0; s < kSizes; ++s) {
                    const pf_tune_entry &e = t.e[c][k][r][s];
                    fprintf(f,
                            "%s    {\"context\": %d, \"kind\": %d, \"r\": %d, \"size_class\": %d, \"variant\": %d, "
                            "\"rows_per_wave\": %d, \"waves_per_group\": %d, \"us\": %.3f}",
                            first ? "" : ",\n", e.context, e.kind, e.r, e.size_class, e.variant, e.rows_per_wave,
                            e.waves_per_group, (double)e.us);
                    first = false;
                }
        }
    fprintf(f, "\n  ]\n}\n");
    const bool ok = fclose(f) == 0;
    return ok ? PF_OK : fail(PF_EINVAL, std::string("cannot write ") + path);
}

pf_status pf_tune_load(const char *path) {
    clear_error();
    if (!path) return fail(PF_EINVAL, "null path");
    FILE *f = fopen(path, "r");
    if (!f) return fail(PF_EINVAL, std::string("cannot read ") + path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    const size_t arr = text.find("\"entries\"");
    if (arr == std::string::npos) return fail(PF_EINVAL, "no \"entries\" in tune file");
    std::vector<pf_tune_entry> es;
    size_t p = text.find('[', arr);
    const size_t stop = p == std::string::npos ? p : text.find(']', p);
    while (p != std::string::npos) {
        const size_t a = text.find('{', p);
        if (a == std::string::npos || a > stop) break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) return fail(PF_EINVAL, "unterminated entry in tune file");
        const std::string obj = text.substr(a, b - a + 1);
        double v[8];
        const char *keys[8] = {"kind", "r", "size_class", "variant", "rows_per_wave", "waves_per_group", "us",
                               "context"};
        for (int i = 0; i < 8; ++i)
            if (!parse_number(obj, keys[i], &v[i])) {
                if (i >= 6) {
                    v[i] = 0.0;  // optional: measured time, context (0: single-image calls)
                } else {
                    return fail(PF_EINVAL, std::string("tune entry without ") + keys[i]);
                }
            }
        pf_tune_entry e;
        e.kind = (int)v[0];
        e.r = (int)v[1];
        e.size_class = (int)v[2];
        e.variant = (int)v[3];
        e.rows_per_wave = (int)v[4];
        e.waves_per_group = (int)v[5];
        e.us = (float)v[6];
        e.context = (int)v[7];
        es.push_back(e);
        p = b + 1;
    }
    // Optional: workgroups per compute unit of batch launches.
    double bpc = kBatchBlocksPerCu;
    const size_t hdr = text.find("\"batch_blocks_per_cu\"");
    if (hdr != std::string::npos && hdr < arr) {
        if (!parse_number(text.substr(hdr, arr - hdr), "batch_blocks_per_cu", &bpc) || bpc < 1 ||
            bpc > kBatchBlocksPerCuMax)
            return fail(PF_EINVAL, "bad batch_blocks_per_cu in tune file");
    }
    const pf_status st = pf_tune_set((int32_t)es.size(), es.data());
    if (st != PF_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.batch_blocks_per_cu = (int)bpc;
    return PF_OK;
}

pf_status pf_tune_batch_blocks(int32_t blocks_per_cu, int32_t *previous) {
    clear_error();
    if (blocks_per_cu < 0 || blocks_per_cu > kBatchBlocksPerCuMax)
        return fail(PF_EINVAL, "blocks_per_cu outside 0.." + std::to_string(kBatchBlocksPerCuMax));
    std::lock_guard<std::mutex> lk(g_mu);
    if (previous) *previous = g_table.batch_blocks_per_cu;
    if (blocks_per_cu > 0) g_table.batch_blocks_per_cu = blocks_per_cu;
    return PF_OK;
}

pf_status pf_autotune(int32_t r_max, int32_t reps, const char *path) {
    clear_error();
    if (r_max < 0 || r_max > PF_R_MAX || reps < 1) return fail(PF_EINVAL, "bad autotune arguments");
    const int bys[] = {8, 16, 32, 64};
    const int wpgs[] = {1, 2, 4, 8};
    hipStream_t s = nullptr;
    hipError_t he = hipStreamCreate(&s);
    if (he != hipSuccess) return fail_hip(he, "stream");
    std::vector<pf_tune_entry> out;
    pf_status st = PF_OK;
    // One pair of buffers large enough for every class: 8 rotating sets of
    // 4096 x 4096 floats (1 GiB touched per rotation, four times what the
    // 256 MB last-level cache holds, so timed reads come from HBM).
    const size_t big = (size_t)4096 * 4096;
    const int nrot = 8;
    float *in = nullptr, *outb = nullptr, *filt = nullptr;
    if ((he = hipMalloc(&in, big * 4 * nrot)) != hipSuccess || (he = hipMalloc(&outb, big * 4 * nrot)) != hipSuccess ||
        (he = hipMalloc(&filt, 4096)) != hipSuccess) {
        st = fail_hip(he, "autotune allocation");
    } else {
        // Timing data: pseudo-random pixels in [0, 1) and small taps. All-zero
        // buffers time markedly faster on MI355X than real data, and would
        // steer the table.
        std::vector<float> host(big);
        uint32_t x = 0x9e3779b9u;
        for (size_t i = 0; i < big; ++i) {
            x ^= x << 13;
            x ^= x >> 17;
            x ^= x << 5;
            host[i] = (float)(x >> 8) * (1.0f / 16777216.0f);
        }
        for (int i = 0; i < nrot && he == hipSuccess; ++i)
            he = hipMemcpy(in + (size_t)i * big, host.data(), big * 4, hipMemcpyHostToDevice);
        std::vector<float> taps(1024, 1.0f / 17.0f);
        if (he == hipSuccess) he = hipMemcpy(filt, taps.data(), 4096, hipMemcpyHostToDevice);
        if (he != hipSuccess) st = fail_hip(he, "autotune data upload");
    }
    // A candidate replaces the best so far only when at least 3% faster, so
    // timing noise does not move the table off its defaults.
    auto better = [](float us, const pf_tune_entry &best) { return best.us == INFINITY || us < 0.97f * best.us; };
    for (int sc = 0; sc < kSizes && st == PF_OK; ++sc) {
        for (int kind = 0; kind < kKinds && st == PF_OK; ++kind) {
            int h, w, n;
            class_shape(sc, kind, &h, &w, &n);
            const size_t px = (size_t)h * w;
            const size_t planes = kind == PF_KIND_U8 ? 3 : 1;
            // rotating buffer sets of one image (uint8: 3 planes)
            const int nb1 = (int)std::max<size_t>(1, std::min<size_t>(64, (big * 4 * nrot) / (px * planes * 4)));
            for (int r = 0; r <= r_max && st == PF_OK; ++r) {
                // ---- single-image calls: every (rows, waves) shape
                const pf_tune_entry dflt = default_entry(PF_TUNE_SINGLE, kind, r, sc);
                pf_tune_entry best = dflt;
                best.us = INFINITY;
                const int var = kind == PF_KIND_SEP ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
                std::vector<std::pair<int, int>> shapes;
                shapes.push_back({dflt.rows_per_wave, dflt.waves_per_group});
                // The uint8 kernel is bound by ALU work and by how evenly its
                // few waves spread over the SIMDs: finer tile heights too.
                std::vector<int> cand(bys, bys + 4);
                if (kind == PF_KIND_U8) cand.insert(cand.end(), {12, 20, 24, 48});
                else
                    for (int by : whole_chunk_heights(r, PF_CHUNK))
                        if (std::find(cand.begin(), cand.end(), by) == cand.end()) cand.push_back(by);
                for (int by : cand)
                    for (int wpg : wpgs)
                        if (by != dflt.rows_per_wave || wpg != dflt.waves_per_group) shapes.push_back({by, wpg});
                auto time_single = [&](int v, int by, int wpg, float *us) -> pf_status {
                    if (kind == PF_KIND_U8) {
                        return time_launch(
                            [&](int i) {
                                const size_t o = (size_t)i * px * planes;
                                return launch_u8(r, v, (const uint8_t *)in + o, (const int8_t *)filt,
                                                 (uint8_t *)outb + o, 3, h, w, 6, by, wpg, s);
                            },
                            nb1, reps, 5, s, us);
                    }
                    return time_launch(
                        [&](int i) {
                            const size_t o = (size_t)i * px;
                            return launch_f32(r, v, false, in + o, filt, filt + (2 * r + 1), outb + o, h, w, by, wpg,
                                              s);
                        },
                        nb1, reps, 5, s, us);
                };
                // A default on another variant (uint8 on the matrix cores) is
                // timed first, so that it keeps its place unless beaten by 3%.
                if (dflt.variant != var) {
                    float us = 0.0f;
                    st = time_single(dflt.variant, dflt.rows_per_wave, dflt.waves_per_group, &us);
                    if (st != PF_OK) break;
                    best.us = us;
                }
                for (const auto &shape : shapes) {
                    float us = 0.0f;
                    st = time_single(var, shape.first, shape.second, &us);
                    if (st != PF_OK) break;
                    if (better(us, best)) {
                        best.variant = var;
                        best.rows_per_wave = shape.first;
                        best.waves_per_group = shape.second;
                        best.us = us;
                    }
                }
                // uint8 on the matrix cores: its own shapes (16-row wave tiles).
                if (st == PF_OK && kind == PF_KIND_U8 && u8_variant_ok(PF_VAR_MFMA, r, 16, 1)) {
                    for (int by : {16, 32, 48, 64}) {
                        for (int wpg : wpgs) {
                            if (!u8_variant_ok(PF_VAR_MFMA, r, by, wpg)) continue;
                            float us = 0.0f;
                            st = time_single(PF_VAR_MFMA, by, wpg, &us);
                            if (st != PF_OK) break;
                            if (better(us, best)) {
                                best.variant = PF_VAR_MFMA;
                                best.rows_per_wave = by;
                                best.waves_per_group = wpg;
                                best.us = us;
                            }
                        }
                        if (st != PF_OK) break;
                    }
                }
                // The variant axis: a separable filter may run as 2D taps.
                if (st == PF_OK && kind == PF_KIND_SEP && r <= PF_SEP_DIRECT_R_MAX) {
                    float us = 0.0f;
                    st = time_single(PF_VAR_SEP_DIRECT, best.rows_per_wave, best.waves_per_group, &us);
                    if (st == PF_OK && better(us, best)) {
                        best.variant = PF_VAR_SEP_DIRECT;
                        best.us = us;
                    }
                }
                if (st != PF_OK) break;
                out.push_back(best);
                // ---- batch kernel: tile heights, on a batch of n class images
                if (kind == PF_KIND_U8 || r > PF_BATCH_R_MAX) continue;
                pf_tune_entry bb = default_entry(PF_TUNE_BATCH, kind, r, sc);
                bb.us = INFINITY;
                for (int by : {bb.rows_per_wave, 8, 32, 64}) {
                    float us = 0.0f;
                    st = time_batch_class(kind, r, h, w, n, by, in, outb, filt, reps, s, &us);
                    if (st != PF_OK) break;
                    if (better(us, bb)) {
                        bb.rows_per_wave = by;
                        bb.us = us;
                    }
                }
                if (st == PF_OK) out.push_back(bb);
            }
        }
    }
    (void)hipStreamSynchronize(s);
    if (in) (void)hipFree(in);
    if (outb) (void)hipFree(outb);
    if (filt) (void)hipFree(filt);
    (void)hipStreamDestroy(s);
    if (st != PF_OK) return st;
    // Keys not measured (r > r_max) keep what they had.
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const pf_tune_entry &e : out) g_table.e[e.context][e.kind][e.r][e.size_class] = e;
    }
    if (path) return pf_tune_save(path);
    return PF_OK;
}

pf_status pf_batch_autotune(int32_t n, const int32_t *__restrict h, const int32_t *__restrict w,
                            const int32_t *__restrict r, const int32_t *__restrict kind,
                            const int64_t *__restrict pix_off, const int64_t *__restrict filt_off, int64_t npix,
                            int64_t nfilt, const float *in, const float *filt, float *out, int32_t reps,
                            const char *path) {
    clear_error();
    if (reps < 1) return fail(PF_EINVAL, "reps must be >= 1");
    if (n < 1 || !h || !w || !r || !kind) return fail(PF_EINVAL, "bad batch description");
    hipStream_t s = nullptr;
    hipError_t he = hipStreamCreate(&s);
    if (he != hipSuccess) return fail_hip(he, "stream");
    // Median time of `reps` replays of a plan built from the active table.
    auto measure = [&](float *us) -> pf_status {
        pf_batch_plan *plan = nullptr;
        pf_status st = pf_batch_plan_create(n, h, w, r, kind, pix_off, filt_off, npix, nfilt, 0, &plan);
        if (st) return st;
        st = time_launch([&](int) -> hipError_t {
            return pf_batch_plan_run(plan, npix, nfilt, in, filt, out, s) == PF_OK ? hipSuccess : hipErrorLaunchFailure;
        }, 1, reps, 5, s, us);
        (void)hipStreamSynchronize(s);
        pf_batch_plan_destroy(plan);
        return st;
    };
    // The batch-context keys (kind, radius, size class) this batch uses.
    std::vector<std::array<int, 3>> keys;
    {
        bool seen[2][PF_R_MAX + 1][kSizes] = {};
        for (int i = 0; i < n; ++i) {
            if ((kind[i] != PF_KIND_2D && kind[i] != PF_KIND_SEP) || r[i] < 0 || r[i] > PF_BATCH_R_MAX || h[i] < 1 ||
                w[i] < 1) {
                (void)hipStreamDestroy(s);
                return fail(PF_EINVAL, "bad image " + std::to_string(i));
            }
            bool &b = seen[kind[i]][r[i]][size_class((int64_t)h[i] * w[i])];
            if (!b) keys.push_back({kind[i], r[i], size_class((int64_t)h[i] * w[i])});
            b = true;
        }
        std::sort(keys.begin(), keys.end());
    }
    // A joint grid first: workgroups per compute unit x one tile height for
    // every key the batch uses (the two interact: the grid sets how many
    // tiles are in flight, the tile height how many tiles there are). The
    // best point is kept outright.
    auto set_all = [&](int by) {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto &k : keys) g_table.e[PF_TUNE_BATCH][k[0]][k[1]][k[2]].rows_per_wave = by;
    };
    float best = INFINITY;
    int best_bpc = 1, best_by = 16;
    pf_status st = PF_OK;
    for (int bpc = 1; bpc <= 4 && st == PF_OK; ++bpc) {
        for (int by : {8, 16, 32, 64}) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_table.batch_blocks_per_cu = bpc;
            }
            set_all(by);
            float us = 0.0f;
            st = measure(&us);
            if (st != PF_OK) break;
            if (us < best) {
                best = us;
                best_bpc = bpc;
                best_by = by;
            }
        }
    }
    if (st == PF_OK) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.batch_blocks_per_cu = best_bpc;
    }
    set_all(best_by);
    // Then coordinate descent over the batch-context keys the batch uses, one
    // key at a time: a new tile height is kept only when the whole batch gets
    // at least 3% faster. Single-image entries are not touched.
    for (const auto &k : keys) {
        if (st != PF_OK) break;
        std::vector<int> bys = {8, 16, 32, 64};
        for (int by : whole_chunk_heights(k[1], PF_BATCH_CHUNK))
            if (std::find(bys.begin(), bys.end(), by) == bys.end()) bys.push_back(by);
        for (int by : bys) {
            int keep = 0;
            {
                std::lock_guard<std::mutex> lk(g_mu);
                pf_tune_entry &e = g_table.e[PF_TUNE_BATCH][k[0]][k[1]][k[2]];
                if (e.rows_per_wave == by) continue;
                keep = e.rows_per_wave;
                e.rows_per_wave = by;
            }
            float us = 0.0f;
            st = measure(&us);
            if (st == PF_OK && us < 0.97f * best) {
                best = us;
            } else {
                std::lock_guard<std::mutex> lk(g_mu);
                g_table.e[PF_TUNE_BATCH][k[0]][k[1]][k[2]].rows_per_wave = keep;
            }
            if (st != PF_OK) break;
        }
    }
    (void)hipStreamDestroy(s);
    if (st != PF_OK) return st;
    {
        // Each key the batch used records the tuned batch's time.
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto &k : keys) g_table.e[PF_TUNE_BATCH][k[0]][k[1]][k[2]].us = best;
    }
    if (path) return pf_tune_save(path);
    return PF_OK;
}

}  // extern "C"
