// Chains of 2D filter passes fused per tile, under four border rules.
//
// A chain applies the same (2r+1)^2 filter `passes` times; pass p reads the
// FP32 image pass p-1 produced, with that image extended past its edges by
// the border rule. Composing several stencil passes into one kernel is the
// cross-component optimisation the paper motivates (Sec. II), for the
// image-processing and fluid-dynamics stencil domains it names (Sec. I);
// every pass keeps the independent-iteration semantics of Sec. II-B.3.
//
// Design (time tiling in LDS): a workgroup owns a 64 x 32 output tile. It
// loads the tile plus a halo of H = r * passes rows and columns once from
// HBM, border-extended on load. Pass p computes, from the LDS image of pass
// p-1, every in-image position within H - p*r of the tile, then writes the
// border extension of its own result into the out-of-image positions of
// that region (interior tiles have none). Reads of a pass therefore never
// need index arithmetic for borders, and only the last pass goes to HBM:
// 8 bytes of HBM traffic per pixel for the whole chain instead of 8 per
// pass. The price is recomputing the halo ring, which shrinks by r per
// pass.
//
// Arithmetic per output: taps in definition order (dy outer, dx inner,
// ascending), one FMA per tap, or with EXACT a separate FP32 multiply and
// add (built with -ffp-contract=off), which reproduces the sequential
// program bit for bit at every pass.
#include "dev_common.h"
#include "pf_internal.h"

namespace pf {
namespace chain {

constexpr int kTileX = 64, kTileY = 32, kThreads = 256;

// Source index of position i of an axis of n elements under a border rule;
// -1 where the rule reads a zero.
__device__ __forceinline__ int border_index(int i, int n, int border) {
    if (i >= 0 && i < n) return i;
    if (border == PF_BORDER_CLAMP) return i < 0 ? 0 : n - 1;
    if (border == PF_BORDER_ZERO) return -1;
    if (border == PF_BORDER_REFLECT) {  // period 2n, edge repeated: d c b a | a b c d | d c b a
        const int p = 2 * n;
        int m = i % p;
        if (m < 0) m += p;
        return m < n ? m : p - 1 - m;
    }
    if (n == 1) return 0;  // PF_BORDER_MIRROR: period 2n-2, edge not repeated
    const int p = 2 * n - 2;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - m;
}

// Workgroup barrier that orders LDS only (a plain __syncthreads() also
// waits for every global access in flight).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool EXACT>
__device__ __forceinline__ float madd(float wgt, float x, float acc) {
    if constexpr (EXACT) {
        const float prod = wgt * x;
        return acc + prod;
    } else {
        return __builtin_fmaf(wgt, x, acc);
    }
}


// LDS layout: one image of (kTileY + 2H) rows and `pitch` floats per row.
// Image column ox (= x0 - H) sits at buffer column pad(R), a multiple of 4
// that is >= R, so the 4-output task at any 4-aligned buffer column c reads
// its window [c - R, c + 3 + R] as 16-byte aligned LDS vectors starting at
// c - pad(R), and consecutive lanes read consecutive 16-byte blocks (no
// bank conflicts).
__host__ __device__ constexpr int lds_pad(int r) { return 4 * ((r + 3) / 4); }
__host__ __device__ constexpr int lds_pitch(int r, int halo) {
    return (2 * lds_pad(r) + kTileX + 2 * halo + 4 + 3) / 4 * 4;
}
__host__ __device__ constexpr int lds_rows(int halo) { return kTileY + 2 * halo + 4; }

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

// Linear task index -> (row, column) over a rows x n grid, stepping by
// kThreads without a division per step.
struct Walk {
    int row, col, drow, dcol, n;
    __device__ __forceinline__ Walk(int start, int n_) : n(n_) {
        row = start / n;
        col = start - row * n;
        drow = kThreads / n;
        dcol = kThreads - drow * n;
    }
    __device__ __forceinline__ void next() {
        row += drow;
        col += dcol;
        if (col >= n) {
            col -= n;
            ++row;
        }
    }
};

// Loads the rows x W0 input region at image (oy, ox) into the buffer
// (region column c at buffer column PAD + c). A lane owns region columns
// lane and lane + 64 (W0 <= 64 + 2 * PF_CHAIN_HALO_MAX), so their source
// columns, border-mapped, are found once; wave v takes rows v, v + 4, ...,
// eight rows (up to 16 loads per lane) in flight before any is waited for.
// BORDER: some positions lie outside the image and read through the border
// rule.
template <bool BORDER>
__device__ __forceinline__ void load_region(const float *__restrict__ in, float *buf, int h, int w, int oy, int ox,
                                            int rows, int W0, int pitch, int pad, int border) {
    constexpr int kRows = 8;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool two = lane + 64 < W0;
    int sx0 = ox + lane, sx1 = ox + lane + 64;
    if constexpr (BORDER) {
        sx0 = border_index(sx0, w, border);
        sx1 = border_index(sx1, w, border);
    }
    float *dst = buf + pad + lane;
    for (int r0 = wave; r0 < rows; r0 += 4 * kRows) {
        float v0[kRows], v1[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int r = r0 + 4 * u;
            int sy = oy + r;
            if constexpr (BORDER) sy = border_index(sy, h, border);
            const bool row_ok = r < rows && sy >= 0;
            const float *src = in + (int64_t)sy * w;
            v0[u] = v1[u] = 0.0f;
            if (row_ok && (!BORDER || sx0 >= 0)) v0[u] = src[sx0];
            if (row_ok && two && (!BORDER || sx1 >= 0)) v1[u] = src[sx1];
        }
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int r = r0 + 4 * u;
            if (r >= rows) break;
            dst[r * pitch] = v0[u];
            if (two) dst[r * pitch + 64] = v1[u];
        }
    }
}

// Tasks one thread holds in registers over a pass (a task: 4 x 4 outputs):
// the largest pass region has at most kTileX / 4 + 2 * ceil((H - R) / 4) + 2
// column blocks and (kTileY + 2 (H - R)) / 4 + 1 row blocks, H <=
// PF_CHAIN_HALO_MAX.
constexpr int kMaxTasks = ((kTileX / 4 + 2 * ((PF_CHAIN_HALO_MAX + 3) / 4) + 2) *
                               ((kTileY + 2 * PF_CHAIN_HALO_MAX) / 4 + 1) +
                           kThreads - 1) /
                          kThreads;

// The passes of one tile over its LDS image `buf` (pass 0 already in it):
// buffer row 0 / column pad(R) holds image position (y0 - H, x0 - H).
template <int R, bool EXACT>
__device__ __forceinline__ void tile_passes(float *buf, int pitch, const float *__restrict__ filt,
                                            float *__restrict__ out, int h, int w, int passes, int border, int x0,
                                            int y0, bool interior, int first) {
    constexpr int K = 2 * R + 1;
    constexpr int PAD = lds_pad(R);
    constexpr int NB = 1 + 2 * PAD / 4;  // 16-byte blocks per window row
    const int H = R * passes;
    const int ox = x0 - H, oy = y0 - H;
    const int cx = PAD - ox;  // buffer column of image column x is x + cx
    // The taps, loaded once: read inside the task loop, their scalar loads
    // would share the LDS reads' wait counter and force a full wait in the
    // middle of every task.
    float wk[K * K];
#pragma unroll
    for (int i = 0; i < K * K; ++i) wk[i] = filt[i];
    // A pass with fewer tasks than threads leaves whole waves idle, and each
    // wave of the workgroup runs on its own SIMD: the wave that takes the
    // pass's first tasks (`first`) therefore moves on past the waves the
    // previous pass used, so that the passes' work spreads over the SIMDs.
    // One LDS image: a pass computes its whole region into registers, and
    // only after a barrier overwrites the previous pass's image with it.
    for (int p = 1; p <= passes; ++p) {
        const bool last = p == passes;
        const int m = (passes - p) * R;  // reach of pass p's region beyond the tile
        const int ylo = max(y0 - m, 0), yhi = min(y0 + kTileY + m, h);
        const int xlo = max(x0 - m, 0), xhi = min(x0 + kTileX + m, w);
        // Tasks: 4 x 4 outputs, rows from ylo in steps of 4, columns at
        // 4-aligned buffer columns covering [xlo, xhi). Window reads stay
        // inside the buffer: columns from c - PAD >= 0 (c >= xlo + cx >= PAD +
        // H - m) to c + 3 + PAD < pitch, rows from ylo - R - oy >= H - m - R
        // >= 0 to at most yhi + 3 + R - oy < rows (4 spare rows). Outputs
        // outside [ylo, yhi) x [xlo, xhi) are computed from whatever the
        // buffer holds there: the last pass does not store them, and task
        // writes back to LDS (rows up to yhi + 2 - oy, columns up to c + 3)
        // stay inside the buffer too.
        const int cb0 = (xlo + cx) >> 2, cb1 = ((xhi - 1 + cx) >> 2) + 1;
        const int ncb = cb1 - cb0, ntask = ((yhi - ylo + 3) >> 2) * ncb;
        float res[kMaxTasks][4][4];
        int at_y[kMaxTasks], at_c[kMaxTasks];
        const int v = (threadIdx.x - 64 * first) & (kThreads - 1);  // this thread's place in task order
        Walk t(v, ncb);
#pragma unroll
        for (int u = 0; u < kMaxTasks; ++u) {
            at_y[u] = ylo + 4 * t.row;
            at_c[u] = 4 * (cb0 + t.col);
            t.next();
            if (v + u * kThreads >= ntask) continue;
            const float *base = buf + (at_y[u] - R - oy) * pitch + (at_c[u] - PAD);
            float acc[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[j][k] = 0.0f;
            // Input row i of the window feeds output rows j = i - dy; rows
            // come in ascending order, so each output takes dy ascending.
#pragma unroll
            for (int i = 0; i < 4 + 2 * R; ++i) {
                float v[4 * NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const f4 q = *reinterpret_cast<const f4 *>(base + i * pitch + 4 * b);
                    v[4 * b] = q.x;
                    v[4 * b + 1] = q.y;
                    v[4 * b + 2] = q.z;
                    v[4 * b + 3] = q.w;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int dy = i - j;
                    if (dy < 0 || dy >= K) continue;
#pragma unroll
                    for (int dx = 0; dx < K; ++dx) {
                        const float wt = wk[dy * K + dx];
#pragma unroll
                        for (int k = 0; k < 4; ++k) acc[j][k] = madd<EXACT>(wt, v[PAD - R + k + dx], acc[j][k]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int k = 0; k < 4; ++k) res[u][j][k] = acc[j][k];
        }
        if (last) {
#pragma unroll
            for (int u = 0; u < kMaxTasks; ++u) {
                if (v + u * kThreads >= ntask) continue;
                const int x = at_c[u] - cx;
                const bool full = x >= xlo && x + 3 < xhi;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int y = at_y[u] + j;
                    if (y >= yhi) continue;
                    float *o = out + (int64_t)y * w;
                    if (full) {
                        // One 16-byte store per row: a wave's lanes cover whole
                        // cache lines (rows need only 4-byte alignment).
                        f4u q;
                        q.x = res[u][j][0];
                        q.y = res[u][j][1];
                        q.z = res[u][j][2];
                        q.w = res[u][j][3];
                        __builtin_nontemporal_store(q, reinterpret_cast<f4u *>(o + x));
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (x + k >= xlo && x + k < xhi) __builtin_nontemporal_store(res[u][j][k], o + x + k);
                    }
                }
            }
            break;
        }
        first = (first + ((ntask + 63) >> 6)) & 3;
        lds_barrier();  // every read of the previous image is done
        // Whole tasks go back to LDS, also their outputs outside the region:
        // those positions lie inside the buffer (the bounds above), and the
        // next pass reads none of them, except out-of-image positions, which
        // the border extension below rewrites first.
#pragma unroll
        for (int u = 0; u < kMaxTasks; ++u) {
            if (v + u * kThreads >= ntask) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                f4 q;
                q.x = res[u][j][0];
                q.y = res[u][j][1];
                q.z = res[u][j][2];
                q.w = res[u][j][3];
                *reinterpret_cast<f4 *>(buf + (at_y[u] + j - oy) * pitch + at_c[u]) = q;
            }
        }
        lds_barrier();
        if (!interior) {
            // Border extension of pass p's image over the out-of-image
            // positions that pass p+1 reads: those of its region within R of
            // the image. Each source lies in the in-image part just written:
            // a rule maps a position within R of an edge to within R of it
            // (m >= R here), or wraps inside an image narrower than a tile,
            // which a single tile covers.
            const int ya = max(y0 - m, -R), yb = min(y0 + kTileY + m, h + R);
            const int xa = max(x0 - m, -R), xb = min(x0 + kTileX + m, w + R);
            Walk f(threadIdx.x, xb - xa);
            for (int i = threadIdx.x; i < (yb - ya) * (xb - xa); i += kThreads, f.next()) {
                const int y = ya + f.row, x = xa + f.col;
                if (y >= 0 && y < h && x >= 0 && x < w) continue;
                const int yy = border_index(y, h, border), xx = border_index(x, w, border);
                buf[(y - oy) * pitch + x + cx] = (yy < 0 || xx < 0) ? 0.0f : buf[(yy - oy) * pitch + xx + cx];
            }
            lds_barrier();
        }
    }
}

template <int R, bool EXACT>
__global__ __launch_bounds__(kThreads) void k_chain_f32(const float *__restrict__ in, const float *__restrict__ filt,
                                                        float *__restrict__ out, int h, int w, int passes, int border,
                                                        int tiles_x, int ntiles) {
    constexpr int PAD = lds_pad(R);
    extern __shared__ float lds[];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int H = R * passes;
    const int pitch = lds_pitch(R, H), rows = lds_rows(H);
    const int W0 = kTileX + 2 * H;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int x0 = tx * kTileX, y0 = ty * kTileY;
    const int ox = x0 - H, oy = y0 - H;
    const bool interior = ox >= 0 && oy >= 0 && x0 + kTileX + H <= w && y0 + kTileY + H <= h;
    // Pass 0: the input region, border-extended.
    if (interior)
        load_region<false>(in, lds, h, w, oy, ox, rows - 4, W0, pitch, PAD, border);
    else
        load_region<true>(in, lds, h, w, oy, ox, rows - 4, W0, pitch, PAD, border);
    __syncthreads();
    tile_passes<R, EXACT>(lds, pitch, filt, out, h, w, passes, border, x0, y0, interior, tile & 3);
}

template <int R, bool EXACT>
hipError_t launch_r(const float *in, const float *filt, float *out, int h, int w, int passes, int border,
                    hipStream_t s) {
    const int H = R * passes;
    const int tiles_x = (w + kTileX - 1) / kTileX, tiles_y = (h + kTileY - 1) / kTileY;
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    if (ntiles > INT32_MAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)lds_rows(H) * lds_pitch(R, H) * sizeof(float);
    hipLaunchKernelGGL((k_chain_f32<R, EXACT>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, in, filt, out, h, w,
                       passes, border, tiles_x, (int)ntiles);
    return hipGetLastError();
}

}  // namespace chain

hipError_t launch_chain(int r, bool exact, const float *in, const float *filt, float *out, int h, int w, int passes,
                        int border, hipStream_t s) {
#define PF_CH(R) \
    return exact ? chain::launch_r<R, true>(in, filt, out, h, w, passes, border, s) \
                 : chain::launch_r<R, false>(in, filt, out, h, w, passes, border, s)
    switch (r) {
        case 0: PF_CH(0);
        case 1: PF_CH(1);
        case 2: PF_CH(2);
        case 3: PF_CH(3);
        case 4: PF_CH(4);
        case 5: PF_CH(5);
        case 6: PF_CH(6);
        case 7: PF_CH(7);
        case 8: PF_CH(8);
        default: return hipErrorInvalidValue;
    }
#undef PF_CH
}

}  // namespace pf
