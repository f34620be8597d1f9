// Radius dispatch for the single-image kernels, the uint8 kernels and the
// batch kernels' entry points.
#include <algorithm>
#include <mutex>

#include "filter_body.h"

namespace pf {

hipError_t launch_f32(int r, int var, bool exact, const float *in, const float *fa, const float *fb, float *out,
                      int h, int w, int by, int wpg, hipStream_t s) {
    switch (r) {
        case 0: return launch_f32_radius<0>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 1: return launch_f32_radius<1>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 2: return launch_f32_radius<2>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 3: return launch_f32_radius<3>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 4: return launch_f32_radius<4>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 5: return launch_f32_radius<5>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 6: return launch_f32_radius<6>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 7: return launch_f32_radius<7>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        case 8: return launch_f32_radius<8>(var, exact, in, fa, fb, out, h, w, by, wpg, s);
        default: return hipErrorInvalidValue;
    }
}

bool u8_variant_ok(int var, int r, int by, int wpg) {
    if (var == PF_VAR_DIRECT) return true;
    return var == PF_VAR_MFMA && r >= 1 && r <= PF_U8_MFMA_R_MAX && by % 16 == 0 && by * wpg <= PF_U8_MFMA_TILE_MAX;
}

hipError_t launch_u8(int r, int var, const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h, int w,
                     int shift, int by, int wpg, hipStream_t s) {
    if (var == PF_VAR_MFMA) {
        if (!u8_variant_ok(var, r, by, wpg)) return hipErrorInvalidValue;
        return launch_u8_mfma(r, in, filt, out, c, h, w, shift, by, wpg, s);
    }
    if (var != PF_VAR_DIRECT) return hipErrorInvalidValue;
    switch (r) {
        case 0: return dev::launch_u8_t<0>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 1: return dev::launch_u8_t<1>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 2: return dev::launch_u8_t<2>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 3: return dev::launch_u8_t<3>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 4: return dev::launch_u8_t<4>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 5: return dev::launch_u8_t<5>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 6: return dev::launch_u8_t<6>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 7: return dev::launch_u8_t<7>(in, filt, out, c, h, w, shift, by, wpg, s);
        case 8: return dev::launch_u8_t<8>(in, filt, out, c, h, w, shift, by, wpg, s);
        default: return hipErrorInvalidValue;
    }
}

void *batch_kernel_fn(int group, bool exact, int mask) {
    if (group != 0) return nullptr;
    switch (mask) {
        case 1: return exact ? batch_fn<0, 1, 1>() : batch_fn<0, 0, 1>();
        case 2: return exact ? batch_fn<0, 1, 2>() : batch_fn<0, 0, 2>();
        default: return exact ? batch_fn<0, 1, 3>() : batch_fn<0, 0, 3>();
    }
}

int batch_grid_limit(int group, bool exact, int mask, int wpg) {
    // Cached per (device, exact, mask, waves per group): the occupancy query
    // is host work that every server batch would otherwise repeat.
    static std::mutex mu;
    static int cache[64][2][4][9] = {};
    const int dev = std::min(std::max(dev_info().device, 0), 63);
    const int m = std::min(std::max(mask, 0), 3), wq = std::min(std::max(wpg, 0), 8);
    {
        std::lock_guard<std::mutex> lk(mu);
        if (group == 0 && cache[dev][exact][m][wq]) return cache[dev][exact][m][wq];
    }
    int blocks = 0;
    void *fn = batch_kernel_fn(group, exact, mask);
    if (!fn ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, wpg * dev::kLanes, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    const int limit = blocks * dev_info().cus;
    if (group == 0) {
        std::lock_guard<std::mutex> lk(mu);
        cache[dev][exact][m][wq] = limit;
    }
    return limit;
}

int batch_grid(int group, bool exact, int mask, int wpg, int64_t ntiles) {
    const int fit = batch_grid_limit(group, exact, mask, wpg);
    const int64_t want = (int64_t)tune_batch_blocks_per_cu() * dev_info().cus;
    const int64_t need = (ntiles + wpg - 1) / wpg;
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, fit), need));
}

hipError_t launch_batch(int group, bool exact, int mask, const BatchImg *imgs, const BatchTask *tasks, int ntasks,
                        int grid, int wpg, const float *in, const float *filt, float *out, hipStream_t s) {
#define PF_LB(G, E, M) launch_batch_g<G, E, M>(imgs, tasks, ntasks, grid, wpg, in, filt, out, s)
    if (group != 0) return hipErrorInvalidValue;
    switch (mask) {
        case 1: return exact ? PF_LB(0, 1, 1) : PF_LB(0, 0, 1);
        case 2: return exact ? PF_LB(0, 1, 2) : PF_LB(0, 0, 2);
        default: return exact ? PF_LB(0, 1, 3) : PF_LB(0, 0, 3);
    }
#undef PF_LB
}

}  // namespace pf
