// Measurement probes: the ALU issue rate and HBM copy rate this device
// reaches with plain kernels, against which the filter kernels' timings are
// read (the filters' rooflines use the published peaks; these say how much
// of a peak a simple kernel of the same instruction or access mix gets).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "pf_internal.h"
#include "pf_probe.h"

namespace pf {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;   // independent dependency chains per lane
constexpr int kProbeUnroll = 16;  // instructions per chain per iteration

// iters x 16 x 8 v_dot4 per lane on 8 independent accumulators.
__global__ __launch_bounds__(kProbeThreads) void k_probe_dot4(int32_t *__restrict__ out, int iters, int b) {
    int a[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = (int)threadIdx.x + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) a[k] = __builtin_amdgcn_sdot4(a[k], b + k, a[k], false);
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += a[k];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// The same shape with v_fma_f32.
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma(float *__restrict__ out, int iters, float b) {
    float a[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = (float)threadIdx.x + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) a[k] = __builtin_fmaf(a[k], b, 0.5f);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += a[k];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;  // 16-byte loads in flight per lane

// Flat copy: each workgroup moves kCopyUnroll x 256 consecutive float4,
// all loads issued before the stores; non-temporal both ways, as the
// filters' loads and stores.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const f4 *__restrict__ in, f4 *__restrict__ out,
                                                              int64_t n4) {
    const int64_t base = (int64_t)blockIdx.x * kCopyUnroll * kProbeThreads + threadIdx.x;
    f4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kProbeThreads;
        v[u] = i < n4 ? __builtin_nontemporal_load(in + i) : f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kProbeThreads;
        if (i < n4) __builtin_nontemporal_store(v[u], out + i);
    }
}

// The last n % 4 floats.
__global__ void k_probe_copy_tail(const float *__restrict__ in, float *__restrict__ out, int64_t from, int64_t n) {
    const int64_t i = from + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace
}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_probe_alu(int32_t op, int32_t blocks, int32_t iters, void *out, void *stream) {
    clear_error();
    if (op != PF_PROBE_DOT4 && op != PF_PROBE_FMA) return fail(PF_EINVAL, "unknown probe");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(PF_EINVAL, "blocks and iters must be in 1..2^20");
    if (!out || (uintptr_t)out % 4) return fail(PF_EINVAL, "out must be a 4-byte aligned device pointer");
    hipStream_t s = (hipStream_t)stream;
    if (op == PF_PROBE_DOT4)
        hipLaunchKernelGGL(k_probe_dot4, dim3(blocks), dim3(kProbeThreads), 0, s, (int32_t *)out, iters, 0x01020304);
    else
        hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kProbeThreads), 0, s, (float *)out, iters, 0.999f);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PF_OK : fail_hip(e, "probe launch");
}

pf_status pf_probe_copy(int64_t n, const float *in, float *out, void *stream) {
    clear_error();
    if (n < 0) return fail(PF_EINVAL, "n must be >= 0");
    if (n == 0) return PF_OK;
    if (!in || !out || (uintptr_t)in % 16 || (uintptr_t)out % 16)
        return fail(PF_EINVAL, "in and out must be 16-byte aligned device pointers");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n4 = n / 4;
    const int64_t per = (int64_t)kCopyUnroll * kProbeThreads;
    if (n4 > 0) {
        const int64_t grid = (n4 + per - 1) / per;
        if (grid > INT32_MAX) return fail(PF_EUNSUPPORTED, "copy too large");
        hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)grid), dim3(kProbeThreads), 0, s, (const f4 *)in, (f4 *)out,
                           n4);
    }
    if (n % 4) hipLaunchKernelGGL(k_probe_copy_tail, dim3(1), dim3(4), 0, s, in, out, 4 * n4, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PF_OK : fail_hip(e, "probe launch");
}

}  // extern "C"
