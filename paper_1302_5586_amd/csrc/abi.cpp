// C ABI entry points for single images, status strings and error text.
//
// Validation follows the paper's coding rules for array parameters
// (Sec. II-B.1): `static N` means at least N elements, so every size must be
// >= 1; `restrict` means distinct arrays never share memory, so an output
// range that overlaps an input range is rejected (PF_EALIAS) rather than
// computed. Nothing is enqueued when validation fails.
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "pf_internal.h"

namespace pf {

static thread_local std::string t_err;

pf_status fail(pf_status s, const std::string &msg) {
    t_err = msg;
    return s;
}

pf_status fail_hip(hipError_t e, const char *what) {
    t_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EDEVICE;
}

void clear_error() { t_err.clear(); }

const DevInfo &dev_info() {
    // One entry per device id; filled on first use with that device current.
    static std::mutex mu;
    static DevInfo infos[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    DevInfo &d = infos[dev];
    if (d.device < 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
            d.cus = p.multiProcessorCount;
            d.arch = p.gcnArchName;
        } else {
            d.cus = 256;
        }
        d.device = dev;
    }
    return d;
}

bool valid_shape(int by, int wpg) {
    const bool by_ok = by >= 4 && by <= 128 && by % 4 == 0;
    const bool wpg_ok = wpg == 1 || wpg == 2 || wpg == 4 || wpg == 8;
    return by_ok && wpg_ok;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

static pf_status check_image(int32_t h, int32_t w, int32_t r) {
    if (h < 1 || w < 1) return fail(PF_EINVAL, "image sizes must be >= 1 (h=" + std::to_string(h) + ", w=" + std::to_string(w) + ")");
    if (r < 0 || r > PF_R_MAX) return fail(PF_EINVAL, "radius " + std::to_string(r) + " outside 0.." + std::to_string(PF_R_MAX));
    if ((int64_t)h * w > (int64_t)INT32_MAX) return fail(PF_EUNSUPPORTED, "image larger than 2^31-1 elements");
    return PF_OK;
}

static pf_status check_f32_bufs(int32_t h, int32_t w, const float *in, const float *out) {
    if (!in || !out) return fail(PF_EINVAL, "null image pointer");
    if (((uintptr_t)in | (uintptr_t)out) % 4) return fail(PF_EINVAL, "FP32 buffers must be 4-byte aligned");
    const size_t bytes = (size_t)h * (size_t)w * sizeof(float);
    if (overlap(in, bytes, out, bytes)) return fail(PF_EALIAS, "input and output overlap (restrict)");
    return PF_OK;
}

// fa: 2D taps or fx; fb: fy (separable kinds only).
static pf_status run_f32(int32_t h, int32_t w, int32_t r, int32_t kind, int var, int by, int wpg, const float *in,
                         const float *fa, const float *fb, float *out, int32_t flags, void *stream) {
    if (flags & ~PF_FLAG_EXACT) return fail(PF_EINVAL, "unknown flags");
    const int k = 2 * r + 1;
    const size_t bytes = (size_t)h * (size_t)w * sizeof(float);
    if (!fa || (kind == PF_KIND_SEP && !fb)) return fail(PF_EINVAL, "null filter pointer");
    if (((uintptr_t)fa | (uintptr_t)fb) % 4) return fail(PF_EINVAL, "filters must be 4-byte aligned");
    if (kind == PF_KIND_2D) {
        if (overlap(fa, (size_t)k * k * sizeof(float), out, bytes)) return fail(PF_EALIAS, "filter and output overlap (restrict)");
    } else {
        if (overlap(fa, k * sizeof(float), out, bytes) || overlap(fb, k * sizeof(float), out, bytes))
            return fail(PF_EALIAS, "filter and output overlap (restrict)");
    }
    hipError_t e = launch_f32(r, var, (flags & PF_FLAG_EXACT) != 0, in, fa, fb, out, h, w, by, wpg, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

}  // namespace pf

using namespace pf;

extern "C" {

const char *pf_status_str(pf_status s) {
    switch (s) {
        case PF_OK: return "PF_OK";
        case PF_EINVAL: return "PF_EINVAL";
        case PF_EALIAS: return "PF_EALIAS";
        case PF_EUNSUPPORTED: return "PF_EUNSUPPORTED";
        case PF_EDEVICE: return "PF_EDEVICE";
        case PF_ENOMEM: return "PF_ENOMEM";
        case PF_EBUDGET: return "PF_EBUDGET";
        case PF_EAGAIN: return "PF_EAGAIN";
        case PF_ETIMEDOUT: return "PF_ETIMEDOUT";
        default: return "PF_UNKNOWN";
    }
}

const char *pf_last_error(void) { return t_err.c_str(); }

const char *pf_version(void) { return "pencilfilter 0.1 gfx950"; }

pf_status pf_filter2d_f32(int32_t h, int32_t w, int32_t r, const float *in, const float *filt, float *out,
                          int32_t flags, void *stream) {
    clear_error();
    pf_status st = check_image(h, w, r);
    if (st) return st;
    if ((st = check_f32_bufs(h, w, in, out))) return st;
    const pf_tune_entry e = tune_lookup(PF_KIND_2D, r, (int64_t)h * w);
    return run_f32(h, w, r, PF_KIND_2D, PF_VAR_DIRECT, e.rows_per_wave, e.waves_per_group, in, filt, nullptr, out, flags,
                   stream);
}

pf_status pf_filter_chain_f32(int32_t h, int32_t w, int32_t r, int32_t passes, int32_t border, const float *in,
                              const float *filt, float *out, int32_t flags, void *stream) {
    clear_error();
    pf_status st = check_image(h, w, r);
    if (st) return st;
    if ((st = check_f32_bufs(h, w, in, out))) return st;
    if (flags & ~PF_FLAG_EXACT) return fail(PF_EINVAL, "unknown flags");
    if (border < PF_BORDER_CLAMP || border > PF_BORDER_MIRROR)
        return fail(PF_EINVAL, "unknown border rule " + std::to_string(border));
    if (passes < 1) return fail(PF_EINVAL, "passes must be >= 1");
    if ((int64_t)r * passes > PF_CHAIN_HALO_MAX)
        return fail(PF_EUNSUPPORTED, "r * passes = " + std::to_string((int64_t)r * passes) + " exceeds " +
                                         std::to_string(PF_CHAIN_HALO_MAX));
    if (!filt) return fail(PF_EINVAL, "null filter pointer");
    if ((uintptr_t)filt % 4) return fail(PF_EINVAL, "filters must be 4-byte aligned");
    const int k = 2 * r + 1;
    if (overlap(filt, (size_t)k * k * sizeof(float), out, (size_t)h * (size_t)w * sizeof(float)))
        return fail(PF_EALIAS, "filter and output overlap (restrict)");
    hipError_t e = launch_chain(r, (flags & PF_FLAG_EXACT) != 0, in, filt, out, h, w, passes, border,
                                (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

static const int64_t kReduceMax = (int64_t)1 << 40;

pf_status pf_sum_workspace(int64_t n, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PF_EINVAL, "null output");
    if (n < 1 || n > kReduceMax) return fail(PF_EINVAL, "n must be in 1..2^40");
    *bytes = sum_workspace_bytes(n);
    return PF_OK;
}

pf_status pf_sum_f32(int64_t n, const float *x, double *out, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (n < 1 || n > kReduceMax) return fail(PF_EINVAL, "n must be in 1..2^40");
    if (!x || !out || !workspace) return fail(PF_EINVAL, "null pointer");
    if ((uintptr_t)x % 4) return fail(PF_EINVAL, "x must be 4-byte aligned");
    if (((uintptr_t)out | (uintptr_t)workspace) % 8) return fail(PF_EINVAL, "out and workspace must be 8-byte aligned");
    const size_t need = sum_workspace_bytes(n);
    if (workspace_bytes < need)
        return fail(PF_EINVAL, "workspace of " + std::to_string(workspace_bytes) + " bytes, " + std::to_string(need) +
                                   " needed");
    const size_t xb = (size_t)n * sizeof(float);
    if (overlap(x, xb, out, 2 * sizeof(double)) || overlap(x, xb, workspace, need) ||
        overlap(out, 2 * sizeof(double), workspace, need))
        return fail(PF_EALIAS, "x, out and workspace must not overlap (restrict)");
    hipError_t e = launch_sum(x, n, out, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

pf_status pf_sum_f32_noalloc(int64_t n, const float *x, double *out, void *stream) {
    clear_error();
    if (n < 1) return fail(PF_EINVAL, "n must be >= 1");
    if (n > sum_noalloc_max())
        return fail(PF_EUNSUPPORTED, "n exceeds the static scratch capacity of " + std::to_string(sum_noalloc_max()) +
                                         " elements (use pf_sum_f32 with a workspace)");
    if (!x || !out) return fail(PF_EINVAL, "null pointer");
    if ((uintptr_t)x % 4) return fail(PF_EINVAL, "x must be 4-byte aligned");
    if ((uintptr_t)out % 8) return fail(PF_EINVAL, "out must be 8-byte aligned");
    if (overlap(x, (size_t)n * sizeof(float), out, 2 * sizeof(double)))
        return fail(PF_EALIAS, "x and out must not overlap (restrict)");
    void *ws = nullptr;
    hipError_t e = sum_scratch(&ws);
    if (e != hipSuccess) return fail_hip(e, "static scratch address");
    e = launch_sum(x, n, out, ws, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

pf_status pf_hist_workspace(int64_t n, size_t *bytes) {
    clear_error();
    if (!bytes) return fail(PF_EINVAL, "null output");
    if (n < 1 || n > kReduceMax) return fail(PF_EINVAL, "n must be in 1..2^40");
    *bytes = hist_workspace_bytes(n);
    return PF_OK;
}

pf_status pf_hist256_u8(int64_t n, const uint8_t *x, int64_t *hist, void *workspace, size_t workspace_bytes,
                        void *stream) {
    clear_error();
    if (n < 1 || n > kReduceMax) return fail(PF_EINVAL, "n must be in 1..2^40");
    if (!x || !hist || !workspace) return fail(PF_EINVAL, "null pointer");
    if ((uintptr_t)hist % 8) return fail(PF_EINVAL, "hist must be 8-byte aligned");
    if ((uintptr_t)workspace % 4) return fail(PF_EINVAL, "workspace must be 4-byte aligned");
    const size_t need = hist_workspace_bytes(n);
    if (workspace_bytes < need)
        return fail(PF_EINVAL, "workspace of " + std::to_string(workspace_bytes) + " bytes, " + std::to_string(need) +
                                   " needed");
    if (overlap(x, (size_t)n, hist, 256 * sizeof(int64_t)) || overlap(x, (size_t)n, workspace, need) ||
        overlap(hist, 256 * sizeof(int64_t), workspace, need))
        return fail(PF_EALIAS, "x, hist and workspace must not overlap (restrict)");
    hipError_t e = launch_hist(x, n, hist, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

pf_status pf_filter2d_f32_border(int32_t h, int32_t w, int32_t r, int32_t border, const float *in, const float *filt,
                                 float *out, int32_t flags, void *stream) {
    if (border == PF_BORDER_CLAMP) return pf_filter2d_f32(h, w, r, in, filt, out, flags, stream);
    return pf_filter_chain_f32(h, w, r, 1, border, in, filt, out, flags, stream);
}

pf_status pf_filter_sep_f32(int32_t h, int32_t w, int32_t r, const float *in, const float *fx, const float *fy,
                            float *out, int32_t flags, void *stream) {
    clear_error();
    pf_status st = check_image(h, w, r);
    if (st) return st;
    if ((st = check_f32_bufs(h, w, in, out))) return st;
    const pf_tune_entry e = tune_lookup(PF_KIND_SEP, r, (int64_t)h * w);
    // The exact flag reproduces the sequential separable program, so it
    // always runs the separable form.
    const bool exact = (flags & PF_FLAG_EXACT) != 0;
    const int var = (!exact && e.variant == PF_VAR_SEP_DIRECT) ? PF_VAR_SEP_DIRECT : PF_VAR_SEPARABLE;
    return run_f32(h, w, r, PF_KIND_SEP, var, e.rows_per_wave, e.waves_per_group, in, fx, fy, out, flags, stream);
}

pf_status pf_filter_f32_shaped(int32_t h, int32_t w, int32_t r, int32_t kind, int32_t variant, int32_t rows_per_wave,
                               int32_t waves_per_group, const float *in, const float *filt, float *out, int32_t flags,
                               void *stream) {
    clear_error();
    pf_status st = check_image(h, w, r);
    if (st) return st;
    if ((st = check_f32_bufs(h, w, in, out))) return st;
    if (kind != PF_KIND_2D && kind != PF_KIND_SEP) return fail(PF_EINVAL, "unknown filter kind");
    if (variant < PF_VAR_DIRECT || variant > PF_VAR_SEP_DIRECT) return fail(PF_EINVAL, "unknown variant");
    if (kind == PF_KIND_2D && variant != PF_VAR_DIRECT) return fail(PF_EINVAL, "a 2D filter runs only as PF_VAR_DIRECT");
    if (kind == PF_KIND_SEP && variant == PF_VAR_DIRECT) variant = PF_VAR_SEP_DIRECT;
    if (variant == PF_VAR_SEP_DIRECT && r > PF_SEP_DIRECT_R_MAX)
        return fail(PF_EUNSUPPORTED, "PF_VAR_SEP_DIRECT runs radii 0.." + std::to_string(PF_SEP_DIRECT_R_MAX));
    if (!valid_shape(rows_per_wave, waves_per_group)) return fail(PF_EINVAL, "unsupported launch shape");
    const float *fb = (kind == PF_KIND_SEP && filt) ? filt + (2 * r + 1) : nullptr;
    return run_f32(h, w, r, kind, variant, rows_per_wave, waves_per_group, in, filt, fb, out, flags, stream);
}

pf_status pf_filter2d_u8(int32_t c, int32_t h, int32_t w, int32_t r, int32_t shift, const uint8_t *in,
                         const int8_t *filt, uint8_t *out, int32_t flags, void *stream) {
    clear_error();
    if (c < 1) return fail(PF_EINVAL, "plane count must be >= 1");
    pf_status st = check_image(h, w, r);
    if (st) return st;
    if ((int64_t)c * h * w > ((int64_t)1 << 40)) return fail(PF_EUNSUPPORTED, "image too large");
    if (shift < 0 || shift > 31) return fail(PF_EINVAL, "shift outside 0..31");
    if (flags != 0) return fail(PF_EINVAL, "unknown flags");
    if (!in || !out || !filt) return fail(PF_EINVAL, "null pointer");
    const size_t bytes = (size_t)c * h * w;
    if (overlap(in, bytes, out, bytes)) return fail(PF_EALIAS, "input and output overlap (restrict)");
    const size_t nf = (size_t)(2 * r + 1) * (2 * r + 1);
    if (overlap(filt, nf, out, bytes)) return fail(PF_EALIAS, "filter and output overlap (restrict)");
    const pf_tune_entry e = tune_lookup(PF_KIND_U8, r, (int64_t)c * h * w);
    hipError_t he =
        launch_u8(r, e.variant, in, filt, out, c, h, w, shift, e.rows_per_wave, e.waves_per_group, (hipStream_t)stream);
    if (he != hipSuccess) return fail_hip(he, "kernel launch");
    return PF_OK;
}

}  // extern "C"
