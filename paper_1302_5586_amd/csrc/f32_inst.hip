// Instantiates the FP32 single-image kernels of one radius (PF_R, set by
// the build) so that radii compile in parallel.
#include "filter_body.h"

#ifndef PF_R
#error "PF_R must be defined"
#endif

namespace pf {

template <>
hipError_t launch_f32_radius<PF_R>(int var, bool exact, const float *in, const float *fa, const float *fb, float *out,
                                   int h, int w, int by, int wpg, hipStream_t s) {
    return exact ? dev::launch_f32_v<PF_R, true>(var, in, fa, fb, out, h, w, by, wpg, s)
                 : dev::launch_f32_v<PF_R, false>(var, in, fa, fb, out, h, w, by, wpg, s);
}

}  // namespace pf
