// Instantiates one persistent batch kernel, selected by the build:
//   PF_GROUP: 0 for radii 0..4 (the only group built);
//   PF_EXACT: 0 fused multiply-add, 1 separate multiply and add;
//   PF_VMASK: bit v set if variant v (PF_VAR_*) is compiled in.
#include "filter_body.h"

#if !defined(PF_GROUP) || !defined(PF_EXACT) || !defined(PF_VMASK)
#error "PF_GROUP, PF_EXACT and PF_VMASK must be defined"
#endif

namespace pf {

namespace {
constexpr int kLo = PF_GROUP == 0 ? 0 : 5;
constexpr int kHi = PF_GROUP == 0 ? 4 : 8;
constexpr bool kExact = PF_EXACT != 0;
}  // namespace

template <>
void *batch_fn<PF_GROUP, PF_EXACT, PF_VMASK>() {
    return (void *)dev::k_batch_f32<kLo, kHi, kExact, PF_VMASK>;
}

template <>
hipError_t launch_batch_g<PF_GROUP, PF_EXACT, PF_VMASK>(const BatchImg *imgs, const BatchTask *tasks, int ntasks,
                                                        int grid, int wpg, const float *in, const float *filt,
                                                        float *out, hipStream_t s) {
    hipLaunchKernelGGL((dev::k_batch_f32<kLo, kHi, kExact, PF_VMASK>), dim3(grid), dim3(wpg * dev::kLanes), 0, s, imgs,
                       tasks, ntasks, in, filt, out);
    return hipGetLastError();
}

}  // namespace pf
