// Reductions next to the filter: the sum (and mean) of an FP32 array and the
// 256-bin histogram of a uint8 array.
//
// The paper's `reduction` directive marks scalars that a loop accumulates
// into, so that the iterations may still run in parallel (Sec. II-B.3), and
// OptiML's `sum` becomes a for loop with such a reduction (Sec. III-B). The
// histogram is the indirect increment A[t[i]]++ of the `independent`
// example (Sec. II-B.3), where t[i] repeats: a reduction per bin.
//
// Reassociating a floating-point sum changes its rounding (the paper's
// reproducibility remark, Sec. III-A). The sum here is reproducible: the
// array is cut into fixed chunks of kChunk elements, each chunk is summed in
// float64 by a fixed pattern (thread t of 256 takes float4 groups t, t +
// 256, ... in order, then a fixed pairwise tree over the 256 threads), and
// the chunk sums are added by the same fixed tree. None of this depends on
// the grid size or on timing, so every call on every device gives the same
// bits. Histogram counts are integers: any order is exact.
//
// Both run as two launches over a caller-provided workspace (chunk partials,
// per-block sub-histograms), so nothing is allocated and nothing needs
// zeroing.
#include <mutex>

#include "dev_common.h"
#include "pf_internal.h"

namespace pf {
namespace red {

constexpr int kThreads = 256;
constexpr int64_t kChunk = 65536;  // elements per chunk partial (fixed: part of the definition of the result)
constexpr int kSumBlocks = 2048;   // most blocks of the partial-sum launch
constexpr int kHistBlocks = 1024;  // most blocks (sub-histograms) of the histogram launch
constexpr int64_t kHistSpan = 1 << 18;  // bytes per histogram block task

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));


// Fixed pairwise tree over the block's 256 values in LDS; returns the total
// in thread 0.
__device__ __forceinline__ double block_tree(double v, double *s) {
    s[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int half = kThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + half];
        __syncthreads();
    }
    return s[0];
}

// partial[c] = sum of chunk c, for the chunks this block takes.
__global__ __launch_bounds__(kThreads) void k_sum_partial(const float *__restrict__ x, int64_t n,
                                                          double *__restrict__ partial, int64_t nchunks) {
    __shared__ double s[kThreads];
    for (int64_t c = xcd_remap(blockIdx.x, gridDim.x); c < nchunks; c += gridDim.x) {
        const int64_t base = c * kChunk;
        const int64_t len = min(kChunk, n - base);
        const float *p = x + base;
        double acc = 0.0;
        if (len == kChunk) {
            // 64 float4 groups per thread; loads in batches of 16 in flight.
#pragma unroll 1
            for (int k0 = 0; k0 < 64; k0 += 16) {
                f4u q[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) q[k] = *reinterpret_cast<const f4u *>(p + 4 * (threadIdx.x + (k0 + k) * kThreads));
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    acc = acc + (double)q[k].x;
                    acc = acc + (double)q[k].y;
                    acc = acc + (double)q[k].z;
                    acc = acc + (double)q[k].w;
                }
            }
        } else {
            // The same order, element by element, stopping at len.
            for (int k = 0; k < 64; ++k) {
                const int64_t g = 4 * ((int64_t)threadIdx.x + (int64_t)k * kThreads);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (g + e < len) acc = acc + (double)p[g + e];
            }
        }
        const double total = block_tree(acc, s);
        if (threadIdx.x == 0) partial[c] = total;
        __syncthreads();
    }
}

// out[0] = sum of the partials (fixed tree), out[1] = out[0] / n.
__global__ __launch_bounds__(kThreads) void k_sum_final(const double *__restrict__ partial, int64_t nchunks, int64_t n,
                                                        double *__restrict__ out) {
    __shared__ double s[kThreads];
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < nchunks; c += kThreads) acc = acc + partial[c];
    const double total = block_tree(acc, s);
    if (threadIdx.x == 0) {
        out[0] = total;
        out[1] = total / (double)n;
    }
}

// sub[b][v]: count of byte value v in the spans block b takes. The block's
// LDS histogram keeps 32 copies of every bin, interleaved so that copy c of
// bin v is word 32 v + c: lane l counts into copy l mod 32, so the atomics
// of a wave fall into distinct banks whatever the data (a plain 256-word
// histogram serialises lanes whose bins share a bank).
constexpr int kCopies = 32;

// Counts the four bytes of a word into a thread's copy of the histogram.
__device__ __forceinline__ void count_word(uint32_t *mine, uint32_t v) {
    atomicAdd(&mine[kCopies * (v & 0xff)], 1u);
    atomicAdd(&mine[kCopies * ((v >> 8) & 0xff)], 1u);
    atomicAdd(&mine[kCopies * ((v >> 16) & 0xff)], 1u);
    atomicAdd(&mine[kCopies * (v >> 24)], 1u);
}

__global__ __launch_bounds__(kThreads) void k_hist_partial(const uint8_t *__restrict__ x, int64_t n,
                                                           uint32_t *__restrict__ sub) {
    __shared__ uint32_t hs[256 * kCopies];
    for (int i = threadIdx.x; i < 256 * kCopies; i += kThreads) hs[i] = 0u;
    __syncthreads();
    uint32_t *mine = hs + (threadIdx.x & (kCopies - 1));
    const int64_t nspan = (n + kHistSpan - 1) / kHistSpan;
    for (int64_t sp = xcd_remap(blockIdx.x, gridDim.x); sp < nspan; sp += gridDim.x) {
        const int64_t base = sp * kHistSpan;
        const int64_t len = min(kHistSpan, n - base);
        const uint8_t *p = x + base;
        if (((uintptr_t)p & 15) == 0) {
            const int64_t nv = len / 16;  // whole 16-byte groups of the span
            const uint4 *q = reinterpret_cast<const uint4 *>(p);
            int64_t i = threadIdx.x;
            // Four 16-byte loads per thread in flight per step.
            for (; i + 3 * kThreads < nv; i += 4 * kThreads) {
                uint4 v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = q[i + k * kThreads];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    count_word(mine, v[k].x);
                    count_word(mine, v[k].y);
                    count_word(mine, v[k].z);
                    count_word(mine, v[k].w);
                }
            }
            for (; i < nv; i += kThreads) {
                const uint4 v = q[i];
                count_word(mine, v.x);
                count_word(mine, v.y);
                count_word(mine, v.z);
                count_word(mine, v.w);
            }
            for (int64_t j = 16 * nv + threadIdx.x; j < len; j += kThreads) atomicAdd(&mine[kCopies * p[j]], 1u);
        } else if (((uintptr_t)p & 3) == 0) {
            const int64_t nw = len / 4;  // whole dwords of the span
            const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
            int64_t i = threadIdx.x;
            // Four dwords per thread in flight per step.
            for (; i + 3 * kThreads < nw; i += 4 * kThreads) {
                uint32_t v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = q[i + k * kThreads];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    atomicAdd(&mine[kCopies * (v[k] & 0xff)], 1u);
                    atomicAdd(&mine[kCopies * ((v[k] >> 8) & 0xff)], 1u);
                    atomicAdd(&mine[kCopies * ((v[k] >> 16) & 0xff)], 1u);
                    atomicAdd(&mine[kCopies * (v[k] >> 24)], 1u);
                }
            }
            for (; i < nw; i += kThreads) {
                const uint32_t v = q[i];
                atomicAdd(&mine[kCopies * (v & 0xff)], 1u);
                atomicAdd(&mine[kCopies * ((v >> 8) & 0xff)], 1u);
                atomicAdd(&mine[kCopies * ((v >> 16) & 0xff)], 1u);
                atomicAdd(&mine[kCopies * (v >> 24)], 1u);
            }
            for (int64_t j = 4 * nw + threadIdx.x; j < len; j += kThreads) atomicAdd(&mine[kCopies * p[j]], 1u);
        } else {
            for (int64_t j = threadIdx.x; j < len; j += kThreads) atomicAdd(&mine[kCopies * p[j]], 1u);
        }
    }
    __syncthreads();
    uint32_t *o = sub + (int64_t)blockIdx.x * 256;
    for (int v = threadIdx.x; v < 256; v += kThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int c = 0; c < kCopies; ++c) t += hs[kCopies * v + ((c + v) & (kCopies - 1))];
        o[v] = t;
    }
}

// hist[v] = sum over blocks of sub[b][v]: one workgroup per bin, its 256
// threads over the blocks, then a tree in LDS (integers: exact in any order).
__global__ __launch_bounds__(kThreads) void k_hist_final(const uint32_t *__restrict__ sub, int nblocks,
                                                         int64_t *__restrict__ hist) {
    __shared__ int64_t s[kThreads];
    const int v = blockIdx.x;
    int64_t acc = 0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) acc += sub[(int64_t)b * 256 + v];
    s[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int half = kThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) s[threadIdx.x] += s[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) hist[v] = s[0];
}

}  // namespace red

int64_t sum_chunks(int64_t n) { return (n + red::kChunk - 1) / red::kChunk; }

size_t sum_workspace_bytes(int64_t n) { return (size_t)sum_chunks(n) * sizeof(double); }

int hist_blocks(int64_t n) {
    const int64_t spans = (n + red::kHistSpan - 1) / red::kHistSpan;
    return (int)std::min<int64_t>(std::max<int64_t>(spans, 1), red::kHistBlocks);
}

size_t hist_workspace_bytes(int64_t n) { return (size_t)hist_blocks(n) * 256 * sizeof(uint32_t); }

// Scratch of pf_sum_f32_noalloc: the chunk partials of sums of up to
// kScratchChunks * kChunk elements, in a file-scope device array (64 KiB on
// each GPU the library runs on, held until the process ends). In host code
// `scratch` names a host-side stand-in, not device memory: host code uses
// only the per-device address that hipGetSymbolAddress returns.
constexpr int64_t kScratchChunks = 8192;
static __device__ __align__(256) double scratch[kScratchChunks];

int64_t sum_noalloc_max() { return kScratchChunks * red::kChunk; }

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
hipError_t sum_scratch(void **ptr) {
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_sum(const float *x, int64_t n, double *out, void *workspace, hipStream_t s) {
    const int64_t nchunks = sum_chunks(n);
    double *partial = static_cast<double *>(workspace);
    const int grid = (int)std::min<int64_t>(nchunks, red::kSumBlocks);
    hipLaunchKernelGGL(red::k_sum_partial, dim3(grid), dim3(red::kThreads), 0, s, x, n, partial, nchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(red::k_sum_final, dim3(1), dim3(red::kThreads), 0, s, partial, nchunks, n, out);
    return hipGetLastError();
}

hipError_t launch_hist(const uint8_t *x, int64_t n, int64_t *hist, void *workspace, hipStream_t s) {
    const int nb = hist_blocks(n);
    uint32_t *sub = static_cast<uint32_t *>(workspace);
    hipLaunchKernelGGL(red::k_hist_partial, dim3(nb), dim3(red::kThreads), 0, s, x, n, sub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(red::k_hist_final, dim3(256), dim3(red::kThreads), 0, s, sub, nb, hist);
    return hipGetLastError();
}

}  // namespace pf
