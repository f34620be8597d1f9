// Tune table and autotuner: profile-based tuning of the launch shape and of
// the variant a separable filter runs as (the paper's compilation flow ends
// in "profile-based iterative compilation and auto-tuning", Sec. II, Fig. 1).
//
// The table is keyed by (kind, radius, size class) and is consulted by the
// single-image calls, batch plans and the server. Results never depend on
// the launch shape (each output's arithmetic is fixed), only on the
// variant, and the variant depends only on the key.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kKinds = 3;  // PF_KIND_2D, PF_KIND_SEP, PF_KIND_U8
constexpr int kSizes = 3;

struct Table {
    pf_tune_entry e[kKinds][PF_R_MAX + 1][kSizes];
};

pf_tune_entry default_entry(int kind, int r, int sc) {
    pf_tune_entry e;
    e.kind = kind;
    e.r = r;
    e.size_class = sc;
    e.variant = (kind == PF_KIND_SEP) ? PF_VAR_SEPARABLE : PF_VAR_DIRECT;
    e.rows_per_wave = sc == 0 ? 8 : (sc == 1 ? 16 : 32);
    e.waves_per_group = 4;
    e.us = 0.0f;
    return e;
}

Table make_default() {
    Table t;
    for (int k = 0; k < kKinds; ++k)
        for (int r = 0; r <= PF_R_MAX; ++r)
            for (int s = 0; s < kSizes; ++s) t.e[k][r][s] = default_entry(k, r, s);
    return t;
}

std::mutex g_mu;
Table g_table = make_default();

bool entry_ok(const pf_tune_entry &e) {
    if (e.kind < 0 || e.kind >= kKinds || e.r < 0 || e.r > PF_R_MAX || e.size_class < 0 || e.size_class >= kSizes)
        return false;
    if (!valid_shape(e.rows_per_wave, e.waves_per_group)) return false;
    // A separable filter runs separable: the persistent batch kernel
    // compiles only the direct and separable bodies, and the table must give
    // single-image calls and batches the same variant for the same key.
    if (e.kind == PF_KIND_SEP) return e.variant == PF_VAR_SEPARABLE;
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
    return g_table.e[kind][r][size_class(pixels)];
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

// Representative image of each size class.
void class_shape(int sc, int *h, int *w) {
    static const int hs[kSizes] = {160, 600, 2048};
    static const int ws[kSizes] = {200, 700, 2048};
    *h = hs[sc];
    *w = ws[sc];
}

}  // namespace

}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_tune_lookup(int32_t kind, int32_t r, int64_t pixels, pf_tune_entry *const __restrict e) {
    clear_error();
    if (!e) return fail(PF_EINVAL, "null output");
    if (kind < 0 || kind >= kKinds || r < 0 || r > PF_R_MAX || pixels < 1) return fail(PF_EINVAL, "bad tune key");
    *e = tune_lookup(kind, r, pixels);
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
        t.e[e.kind][e.r][e.size_class] = e;
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
    fprintf(f, "{\n  \"library\": \"%s\",\n  \"device_arch\": \"%s\",\n  \"entries\": [\n", pf_version(), d.arch.c_str());
    bool first = true;
    for (int k = 0; k < kKinds; ++k)
        for (int r = 0; r <= PF_R_MAX; ++r)
            for (int s = 0; s < kSizes; ++s) {
                const pf_tune_entry &e = t.e[k][r][s];
                fprintf(f, "%s    {\"kind\": %d, \"r\": %d, \"size_class\": %d, \"variant\": %d, \"rows_per_wave\": %d, "
                           "\"waves_per_group\": %d, \"us\": %.3f}",
                        first ? "" : ",\n", e.kind, e.r, e.size_class, e.variant, e.rows_per_wave, e.waves_per_group,
                        (double)e.us);
                first = false;
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
        double v[7];
        const char *keys[7] = {"kind", "r", "size_class", "variant", "rows_per_wave", "waves_per_group", "us"};
        for (int i = 0; i < 7; ++i)
            if (!parse_number(obj, keys[i], &v[i])) {
                if (i == 6) {
                    v[6] = 0.0;
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
        es.push_back(e);
        p = b + 1;
    }
    return pf_tune_set((int32_t)es.size(), es.data());
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
    for (int sc = 0; sc < kSizes && st == PF_OK; ++sc) {
        int h, w;
        class_shape(sc, &h, &w);
        const size_t px = (size_t)h * w;
        // Rotate buffers so that at least 512 MiB is touched per rotation:
        // the 256 MB last-level cache cannot serve the large class.
        const int nbuf = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)512 << 20) / (px * 8) + 1));
        float *in = nullptr, *outb = nullptr, *filt = nullptr;
        if ((he = hipMalloc(&in, px * 4 * nbuf)) != hipSuccess || (he = hipMalloc(&outb, px * 4 * nbuf)) != hipSuccess ||
            (he = hipMalloc(&filt, 4096)) != hipSuccess) {
            st = fail_hip(he, "autotune allocation");
        } else {
            (void)hipMemsetAsync(in, 0, px * 4 * nbuf, s);
            (void)hipMemsetAsync(filt, 0, 4096, s);
            for (int kind = 0; kind < kKinds && st == PF_OK; ++kind) {
                for (int r = 0; r <= r_max && st == PF_OK; ++r) {
                    pf_tune_entry best = default_entry(kind, r, sc);
                    best.us = INFINITY;
                    const int nvars = 1;
                    for (int vi = 0; vi < nvars && st == PF_OK; ++vi) {
                        const int var = kind == PF_KIND_SEP ? (vi == 0 ? PF_VAR_SEPARABLE : PF_VAR_SEP_DIRECT) : PF_VAR_DIRECT;
                        for (int by : bys)
                            for (int wpg : wpgs) {
                                if (st != PF_OK) break;
                                float us = 0.0f;
                                if (kind == PF_KIND_U8) {
                                    // uint8: 3 planes of the class shape, bytes fit in the same buffers
                                    const uint8_t *ib = (const uint8_t *)in;
                                    uint8_t *ob = (uint8_t *)outb;
                                    const size_t plane3 = 3 * px;
                                    const int nb8 = (int)std::max<size_t>(1, (px * 4 * nbuf) / plane3);
                                    st = time_launch(
                                        [&](int i) {
                                            return launch_u8(r, ib + (size_t)i * plane3, (const int8_t *)filt,
                                                             ob + (size_t)i * plane3, 3, h, w, 6, by, wpg, s);
                                        },
                                        std::min(nb8, nbuf), reps, 3, s, &us);
                                } else {
                                    st = time_launch(
                                        [&](int i) {
                                            return launch_f32(r, var, false, in + (size_t)i * px, filt,
                                                              filt + (2 * r + 1), outb + (size_t)i * px, h, w, by, wpg, s);
                                        },
                                        nbuf, reps, 3, s, &us);
                                }
                                if (st == PF_OK && us < best.us) {
                                    best.variant = var;
                                    best.rows_per_wave = by;
                                    best.waves_per_group = wpg;
                                    best.us = us;
                                }
                            }
                    }
                    out.push_back(best);
                }
            }
        }
        (void)hipStreamSynchronize(s);
        if (in) (void)hipFree(in);
        if (outb) (void)hipFree(outb);
        if (filt) (void)hipFree(filt);
    }
    (void)hipStreamDestroy(s);
    if (st != PF_OK) return st;
    // Keys not measured (r > r_max) keep their defaults.
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const pf_tune_entry &e : out) g_table.e[e.kind][e.r][e.size_class] = e;
    }
    if (path) return pf_tune_save(path);
    return PF_OK;
}

}  // extern "C"
