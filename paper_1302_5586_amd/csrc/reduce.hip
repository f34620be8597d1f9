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

// Sum of one chunk p[0 .. len) (len <= kChunk) by the fixed pattern: thread
// t takes float4 groups t, t + 256, ... in order, then the block tree. The
// total is returned in thread 0. Every caller (single arrays and server
// batches) sums a chunk with this function, so a chunk's bits never depend
// on which launch computed it.
__device__ __forceinline__ double chunk_sum(const float *__restrict__ p, int64_t len, double *s) {
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
    return block_tree(acc, s);
}

// partial[c] = sum of chunk c, for the chunks this block takes.
__global__ __launch_bounds__(kThreads) void k_sum_partial(const float *__restrict__ x, int64_t n,
                                                          double *__restrict__ partial, int64_t nchunks) {
    __shared__ double s[kThreads];
    for (int64_t c = xcd_remap(blockIdx.x, gridDim.x); c < nchunks; c += gridDim.x) {
        const int64_t base = c * kChunk;
        const double total = chunk_sum(x + base, min(kChunk, n - base), s);
        if (threadIdx.x == 0) partial[c] = total;
        __syncthreads();
    }
}

// out[0] = sum of the partials (fixed tree), out[1] = out[0] / n.
__device__ __forceinline__ void final_sum(const double *__restrict__ partial, int64_t nchunks, int64_t n,
                                          double *__restrict__ out, double *s) {
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < nchunks; c += kThreads) acc = acc + partial[c];
    const double total = block_tree(acc, s);
    if (threadIdx.x == 0) {
        out[0] = total;
        out[1] = total / (double)n;
    }
}

__global__ __launch_bounds__(kThreads) void k_sum_final(const double *__restrict__ partial, int64_t nchunks, int64_t n,
                                                        double *__restrict__ out) {
    __shared__ double s[kThreads];
    final_sum(partial, nchunks, n, out, s);
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

// Counts the bytes p[0 .. len) into the calling thread's copy of the block
// histogram: 16-byte loads where p is 16-byte aligned (four per thread in
// flight), dwords where it is 4-byte aligned, bytes otherwise.
__device__ __forceinline__ void count_span(const uint8_t *__restrict__ p, int64_t len, uint32_t *mine) {
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
            for (int k = 0; k < 4; ++k) count_word(mine, v[k]);
        }
        for (; i < nw; i += kThreads) count_word(mine, q[i]);
        for (int64_t j = 4 * nw + threadIdx.x; j < len; j += kThreads) atomicAdd(&mine[kCopies * p[j]], 1u);
    } else {
        for (int64_t j = threadIdx.x; j < len; j += kThreads) atomicAdd(&mine[kCopies * p[j]], 1u);
    }
}

// o[v] = the block histogram's count of value v (its 32 copies added).
__device__ __forceinline__ void fold_copies(const uint32_t *hs, uint32_t *__restrict__ o) {
    for (int v = threadIdx.x; v < 256; v += kThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int c = 0; c < kCopies; ++c) t += hs[kCopies * v + ((c + v) & (kCopies - 1))];
        o[v] = t;
    }
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
        count_span(x + base, min(kHistSpan, n - base), mine);
    }
    __syncthreads();
    fold_copies(hs, sub + (int64_t)blockIdx.x * 256);
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

// ---- many arrays in one launch (server batches) -----------------------------
// Task t of a batch is part `part` (a chunk of kChunk floats for a sum, a
// span of kHistSpan bytes for a histogram) of request `req`; its partial
// goes to slot reqs[req].first + part of the batch workspace. Each part is
// reduced by the same device function as in the single-array kernels, so a
// request's result is bit for bit that of pf_sum_f32 / pf_hist256_u8 on the
// same array, whichever batch it lands in.

__global__ __launch_bounds__(kThreads) void k_sum_partial_multi(const ReduceReq *__restrict__ reqs,
                                                                const ReduceTask *__restrict__ tasks, int ntasks,
                                                                double *__restrict__ partial) {
    __shared__ double s[kThreads];
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntasks; t += gridDim.x) {
        const ReduceTask tk = tasks[t];
        const ReduceReq q = reqs[tk.req];
        const int64_t base = (int64_t)tk.part * kChunk;
        const double total = chunk_sum(global_ptr<const float>(q.in) + base, min(kChunk, q.n - base), s);
        if (threadIdx.x == 0) partial[q.first + tk.part] = total;
        __syncthreads();
    }
}

// One workgroup per sum request (ids lists them).
__global__ __launch_bounds__(kThreads) void k_sum_final_multi(const ReduceReq *__restrict__ reqs,
                                                              const int32_t *__restrict__ ids,
                                                              const double *__restrict__ partial) {
    __shared__ double s[kThreads];
    const ReduceReq q = reqs[ids[blockIdx.x]];
    final_sum(partial + q.first, (q.n + kChunk - 1) / kChunk, q.n, global_ptr<double>(q.out), s);
}

__global__ __launch_bounds__(kThreads) void k_hist_partial_multi(const ReduceReq *__restrict__ reqs,
                                                                 const ReduceTask *__restrict__ tasks, int ntasks,
                                                                 uint32_t *__restrict__ sub) {
    __shared__ uint32_t hs[256 * kCopies];
    uint32_t *mine = hs + (threadIdx.x & (kCopies - 1));
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntasks; t += gridDim.x) {
        const ReduceTask tk = tasks[t];
        const ReduceReq q = reqs[tk.req];
        for (int i = threadIdx.x; i < 256 * kCopies; i += kThreads) hs[i] = 0u;
        __syncthreads();
        const int64_t base = (int64_t)tk.part * kHistSpan;
        count_span(global_ptr<const uint8_t>(q.in) + base, min(kHistSpan, q.n - base), mine);
        __syncthreads();
        fold_copies(hs, sub + (q.first + tk.part) * 256);
        __syncthreads();
    }
}

// Workgroup (v, j): bin v of histogram request ids[j], summed over its spans.
__global__ __launch_bounds__(kThreads) void k_hist_final_multi(const ReduceReq *__restrict__ reqs,
                                                               const int32_t *__restrict__ ids,
                                                               const uint32_t *__restrict__ sub) {
    __shared__ int64_t s[kThreads];
    const int v = blockIdx.x;
    const ReduceReq q = reqs[ids[blockIdx.y]];
    const int64_t nparts = (q.n + kHistSpan - 1) / kHistSpan;
    int64_t acc = 0;
    for (int64_t b = threadIdx.x; b < nparts; b += kThreads) acc += sub[(q.first + b) * 256 + v];
    s[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int half = kThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) s[threadIdx.x] += s[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) global_ptr<int64_t>(q.out)[v] = s[0];
}

}  // namespace red

int64_t reduce_parts(int op, int64_t n) {
    return op == PF_OP_SUM_F32 ? (n + red::kChunk - 1) / red::kChunk : (n + red::kHistSpan - 1) / red::kHistSpan;
}

hipError_t launch_reduce_batch(const ReduceReq *reqs, const int32_t *sum_ids, int nsum, const ReduceTask *sum_tasks,
                               int n_sum_tasks, const int32_t *hist_ids, int nhist, const ReduceTask *hist_tasks,
                               int n_hist_tasks, double *partial, uint32_t *sub, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (nsum > 0) {
        const int grid = std::min(n_sum_tasks, red::kSumBlocks);
        hipLaunchKernelGGL(red::k_sum_partial_multi, dim3(grid), dim3(red::kThreads), 0, s, reqs, sum_tasks,
                           n_sum_tasks, partial);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(red::k_sum_final_multi, dim3(nsum), dim3(red::kThreads), 0, s, reqs, sum_ids, partial);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (nhist > 0) {
        const int grid = std::min(n_hist_tasks, red::kHistBlocks);
        hipLaunchKernelGGL(red::k_hist_partial_multi, dim3(grid), dim3(red::kThreads), 0, s, reqs, hist_tasks,
                           n_hist_tasks, sub);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(red::k_hist_final_multi, dim3(256, nhist), dim3(red::kThreads), 0, s, reqs, hist_ids, sub);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return e;
}

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
