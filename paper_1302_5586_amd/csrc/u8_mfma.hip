// The uint8 filter on the int8 matrix cores (radius 1..PF_U8_MFMA_R_MAX = 8).
//
// At a 7 x 7 filter the uint8 path does 49 multiply-adds per byte read, far
// more than v_dot4 can issue per byte of HBM bandwidth, so the v_dot4
// kernel is bound by VALU issue. Here the sums go to v_mfma_i32_16x16x64_i8
// instead, as a contraction per 16 x 16 block of outputs:
//
//   out[y][x0 + i] = sum over tap row dy and byte column c of
//                    T[i][(dy, c)] * P[(dy, c)][y],
//
// P[(dy, c)][y] = pixel (row y + dy - r, column x0 - 8 + c) of the image,
// c = 0..31, and T the filter laid out as a Toeplitz band:
// T[i][(dy, c)] = f[dy][c - i - 8 + r] where that tap exists, else 0 (the
// taps of output column i sit at c = i + 8 - r .. i + 8 + r, inside 0..31
// for every r <= 8). One
// MFMA k-step of 64 bytes covers two tap rows, so a 2r+1 filter takes r+1
// steps (the last one with a zero tap row when 2r+1 is odd). Each output
// is its definition's sum of integer products, computed exactly in int32,
// so the result is the sequential program's bit for bit whatever the order
// of the terms.
//
// Operand layout (the same byte layout for A and B, so the k order inside
// a step need not be the hardware's): lane l supplies row or column l % 16
// and the 16 bytes of group g = l / 16 of the step, here tap row 2s + g/2
// and byte columns 16 (g % 2) .. +15. Lane l of the 16 x 16 int32 result
// holds column l % 16 (the output row) and rows 4 (l / 16) .. +3 (four
// adjacent output columns), which it packs into one dword; the wave's
// dwords go through LDS so that each lane stores 16 contiguous bytes.
//
// A workgroup owns a tile of 128 output columns and waves x rows-per-wave
// output rows. It stages the tile's input rows (clamped at the image edges,
// biased by -128 to fit the signed operand) and the zero-padded filter rows
// in LDS; each lane assembles its band entries from the latter once, and
// each wave reads its B operands with 16-byte LDS loads, eight column
// blocks at a time. The bias is added back exactly as 128 * sum(weights),
// the initial value of every accumulator.
#include "filter_body.h"

namespace pf {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMfmaN = 16;                    // output rows and columns of one MFMA block
// Column blocks per workgroup tile: 8, so that every output row piece a
// tile stores is a whole 128-byte line (tiles of 4 blocks wrote 64-byte
// halves, 1.33x the output bytes, and took 6.6 us against 6.1 us at 1080p
// RGB, 7 x 7).
constexpr int kMfmaBlocks = 8;
constexpr int kMfmaTileW = kMfmaN * kMfmaBlocks;  // output columns of a workgroup tile
constexpr int kMfmaLeft = 8;                  // staged columns left of the tile
constexpr int kMfmaRow = kMfmaTileW + 16;     // LDS bytes per staged row: columns x0 - 8 .. x0 + W + 7
constexpr int kMfmaGran = 8;                  // bytes a lane stages per row (edge tiles)
constexpr int kMfmaFill = kMfmaRow / kMfmaGran;  // lanes per staged row: every byte of it
constexpr int kMfmaStage = 8;                 // staged loads a thread has in flight at once
static_assert(kMfmaRow % kMfmaGran == 0, "whole granules per staged row");

constexpr int kTapRow = 64;                   // LDS bytes per zero-padded filter row
constexpr int kTapOff = 32;                   // byte of tap 0 in a padded row

template <int R>
constexpr int mfma_steps() {
    return R + 1;
}

// LDS bytes of a workgroup tile `tile_rows` high: the padded filter rows
// (2 per step), the staged rows (tile_rows + 2r + 1: the last one only
// meets zero taps), then 16 output rows per wave.
template <int R>
constexpr int mfma_lds_bytes(int tile_rows, int waves) {
    return 2 * mfma_steps<R>() * kTapRow + (tile_rows + 2 * R + 1) * kMfmaRow + waves * kMfmaN * kMfmaRow;
}

// The filter rows, zero-padded, in LDS: padded row dy (0 .. 2 steps - 1)
// is kTapRow bytes, byte kTapOff + t = tap t (0 <= t <= 2r) of filter row
// dy, every other byte (and every row dy > 2r) 0. Only dwords kTapOff/4 ..
// +4 of a row hold taps; their threads load the row's taps at fixed offsets
// from one address (all in flight together). Lane 16 g + i then reads the
// 16 bytes of its Toeplitz band entry, taps c - i - 8 + r for c = 16 (g % 2)
// .. +15, as a byte-shifted window of padded row 2s + g/2.
template <int R>
__device__ __forceinline__ void stage_taps(const int8_t *__restrict__ filt, uint32_t *taps, int tid, int nthr) {
    constexpr int K = 2 * R + 1;
    constexpr int DW = kTapRow / 4;
    constexpr int TW = (K + 3) / 4;  // dwords of taps per filter row
    static_assert(TW <= 5, "taps of a row within dwords kTapOff/4 .. +4");
    for (int d = tid; d < 2 * mfma_steps<R>() * DW; d += nthr) {
        const int dy = d / DW, c = d % DW - kTapOff / 4;
        uint32_t v = 0u;
        if (dy < K && c >= 0 && c < TW) {
            const int8_t *frow = filt + dy * K;
            uint32_t tw[TW] = {};
#pragma unroll
            for (int t = 0; t < K; ++t) tw[t >> 2] |= (uint32_t)(uint8_t)frow[t] << (8 * (t & 3));
#pragma unroll
            for (int k = 0; k < TW; ++k) v = c == k ? tw[k] : v;
        }
        taps[d] = v;
    }
}

// Staged row ly = image row clamp(y0 - r + ly), bytes G q .. G q + G - 1 =
// columns x0 - 8 + G q .. (each clamped to the image), minus 128, for G =
// kMfmaGran. Rows 0 .. nrows - 1 and granules 0 .. kMfmaFill - 1: every byte
// a nonzero tap reads. The lanes of a wave stage 64 / kMfmaFill rows per
// pass, lane kMfmaFill k + q granule q of one of them, so the column part of
// every load (clamp, byte selectors) is the lane's own constant. ALIGNED
// (rows 4-byte aligned and w >= G, so w is a multiple of 4 and each dword
// of a granule is either inside the image or wholly left or right of it):
// one G-byte load from the clamped position, each dword of it picked by a
// byte selector (identity inside; a broadcast of the edge byte outside);
// else one byte load per byte, of the clamped column. Loads are
// unconditional (clamped rows) and issued kMfmaStage at a time; `between`
// runs after the first batch is issued, before any of it is written.
template <int R, bool ALIGNED, class F>
__device__ __forceinline__ void stage_rows(const uint8_t *__restrict__ plane, uint8_t *rows, int h, int w, int x0,
                                           int y0, int nrows, int wave, int nwaves, int lane, F &&between) {
    constexpr int G = kMfmaGran, ND = G / 4;
    constexpr int PER = kLanes / kMfmaFill;  // rows per wave per pass
    typedef uint32_t gran_t __attribute__((ext_vector_type(ND)));
    const int lr = lane / kMfmaFill, q = lane - lr * kMfmaFill;
    const bool active = lr < PER;
    const int xc = x0 - kMfmaLeft + G * q;
    uint32_t xa = 0, sel[ND];
    uint32_t xo[ALIGNED ? 1 : G];
    if constexpr (ALIGNED) {
        xa = (uint32_t)clampi(xc, 0, w - G);
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            sel[j] = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) sel[j] |= (uint32_t)(clampi(xc + 4 * j + k, 0, w - 1) - (int)xa) << (8 * k);
        }
        xo[0] = xa;
    } else {
#pragma unroll
        for (int j = 0; j < G; ++j) xo[j] = (uint32_t)clampi(xc + j, 0, w - 1);
    }
    uint8_t *dst = rows + lr * kMfmaRow + G * q;
    const int step = PER * nwaves;
    for (int base = PER * wave; base < nrows; base += kMfmaStage * step) {
        gran_t v[kMfmaStage];
#pragma unroll
        for (int u = 0; u < kMfmaStage; ++u) {
            const int ly = min(base + u * step + lr, nrows - 1);
            const uint32_t roff = (uint32_t)clampi(y0 - R + ly, 0, h - 1) * (uint32_t)w;
            if constexpr (ALIGNED) {
                // Selector values 0..3 pick bytes of the first dword, 4..7
                // bytes of the second.
                typedef uint32_t u2 __attribute__((ext_vector_type(2), aligned(4)));
                const u2 d = *(const u2 *)(plane + (roff + xo[0]));
#pragma unroll
                for (int j = 0; j < ND; ++j) v[u][j] = __builtin_amdgcn_perm(d[1], d[0], sel[j]);
            } else {
#pragma unroll
                for (int j = 0; j < ND; ++j) {
                    uint32_t d = 0u;
#pragma unroll
                    for (int k = 0; k < 4; ++k) d |= (uint32_t)plane[roff + xo[4 * j + k]] << (8 * k);
                    v[u][j] = d;
                }
            }
        }
        if (base == PER * wave) between();
#pragma unroll
        for (int u = 0; u < kMfmaStage; ++u) {
            const int r0 = base + u * step;
            if (active && r0 + lr < nrows) {
                gran_t o;
#pragma unroll
                for (int j = 0; j < ND; ++j) o[j] = v[u][j] ^ 0x80808080u;
                *(gran_t *)(dst + r0 * kMfmaRow) = o;
            }
        }
    }
}

// Staging for a tile whose staged columns all lie inside the image (and
// rows 4-byte aligned): no column clamp, 16 bytes per lane (9 lanes per
// row, 7 rows per wave pass), loads issued 4 at a time. At 1080p RGB, 7 x 7
// (all but the edge tiles) 5.7 us against 6.0 us with the 8-byte staging.
template <int R, class F>
__device__ __forceinline__ void stage_rows_wide(const uint8_t *__restrict__ plane, uint8_t *rows, int h, int w,
                                                int x0, int y0, int nrows, int wave, int nwaves, int lane,
                                                F &&between) {
    constexpr int G = 16, NL = kMfmaRow / G, PER = kLanes / NL, ST = 4;
    static_assert(kMfmaRow % G == 0, "whole 16-byte granules per staged row");
    typedef uint32_t u4a __attribute__((ext_vector_type(4), aligned(4)));
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const int lr = lane / NL, q = lane - lr * NL;
    const bool active = lr < PER;
    const uint32_t xo = (uint32_t)(x0 - kMfmaLeft + G * q);
    uint8_t *dst = rows + lr * kMfmaRow + G * q;
    const int step = PER * nwaves;
    for (int base = PER * wave; base < nrows; base += ST * step) {
        u4 v[ST];
#pragma unroll
        for (int u = 0; u < ST; ++u) {
            const int ly = min(base + u * step + lr, nrows - 1);
            const uint32_t roff = (uint32_t)clampi(y0 - R + ly, 0, h - 1) * (uint32_t)w;
            v[u] = *(const u4a *)(plane + (roff + xo));
        }
        if (base == PER * wave) between();
#pragma unroll
        for (int u = 0; u < ST; ++u) {
            const int r0 = base + u * step;
            if (active && r0 + lr < nrows) *(u4 *)(dst + r0 * kMfmaRow) = v[u] ^ 0x80808080u;
        }
    }
}

// The 4 outputs of a lane's accumulators: arithmetic shift, saturation,
// packed little-endian.
__device__ __forceinline__ uint32_t pack_mfma_u8(const v4i &a, int shift) {
    uint32_t pk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int q = clampi(a[k] >> shift, 0, 255);  // arithmetic shift of a signed int
        asm volatile("" : "+v"(q));             // keep the saturated byte opaque until packed (as in store_u8)
        pk |= (uint32_t)q << (8 * k);
    }
    return pk;
}

// 16 outputs of row y, columns x .. x + 15, as four dwords: one 16-byte
// store when the rows are aligned and all 16 columns are in the image, else
// dword stores (aligned rows: a dword is wholly inside or right of the
// image) or byte stores, each dropped outside the image.
__device__ __forceinline__ void store16_mfma_u8(const __amdgpu_buffer_rsrc_t &rs, int h, int w, int y, int x,
                                                bool aligned, const v4i &v) {
    constexpr uint32_t kDrop = 0x80000000u;
    const uint32_t off = (uint32_t)y * (uint32_t)w + (uint32_t)x;
    if (aligned && x + 16 <= w) {
        __builtin_amdgcn_raw_buffer_store_b128(v, rs, y < h ? off : kDrop, 0, kStoreAux);
    } else if (aligned) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v[k], rs, (y < h && x + 4 * k < w) ? off + 4 * k : kDrop, 0,
                                                  kStoreAux);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)((uint32_t)v[k >> 2] >> (8 * (k & 3))), rs,
                                                 (y < h && x + k < w) ? off + k : kDrop, 0, kStoreAux);
    }
}

// Workgroup tile t of the launch: plane t / tiles_per_plane, tile column
// (t mod tiles_per_plane) mod tiles_x, tile row (t mod tiles_per_plane) /
// tiles_x. Wave v computes rows rpw v .. rpw (v + 1) - 1 of the tile (rpw a
// multiple of 16), 16 rows at a time.
template <int R>
__global__ __launch_bounds__(512) void k_filter_u8_mfma(const uint8_t *__restrict__ in,
                                                        const int8_t *__restrict__ filt, uint8_t *__restrict__ out,
                                                        int h, int w, int shift, int aligned, int rpw, int tiles_x,
                                                        int tiles_per_plane, int ntiles) {
    constexpr int NS = mfma_steps<R>();
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t *taps = (uint32_t *)lds;
    uint8_t *rows = lds + 2 * NS * kTapRow;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;  // whole workgroup
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    const int p = t / tiles_per_plane;
    const int local = t - p * tiles_per_plane;
    const int ty = local / tiles_x;
    const int x0 = (local - ty * tiles_x) * kMfmaTileW;
    const int tile_rows = rpw * (nthr / kLanes);
    const int y0 = ty * tile_rows;
    const int64_t plane = (int64_t)p * h * w;
    const int nstage = min(tile_rows, h - y0) + 2 * R;  // rows whose outputs exist, plus the halo

    const int lane = tid % kLanes;
    const int wave = uniform(tid / kLanes);
    const int nwaves = nthr / kLanes;
    // The taps' loads are issued while the first rows' loads are in flight.
    auto taps_step = [&]() __attribute__((always_inline)) { stage_taps<R>(filt, taps, tid, nthr); };
    if (aligned && x0 >= kMfmaLeft && x0 + kMfmaRow - kMfmaLeft <= w)
        stage_rows_wide<R>(in + plane, rows, h, w, x0, y0, nstage, wave, nwaves, lane, taps_step);
    else if (aligned && w >= kMfmaGran)
        stage_rows<R, true>(in + plane, rows, h, w, x0, y0, nstage, wave, nwaves, lane, taps_step);
    else
        stage_rows<R, false>(in + plane, rows, h, w, x0, y0, nstage, wave, nwaves, lane, taps_step);
    __syncthreads();

    const int m = lane & 15, g = lane >> 4;
    // A operand of step s: 16 bytes of padded row 2s + g/2 from byte pa
    // (10 <= pa <= 48), read as five dwords and shifted by pa mod 4 bytes.
    const int pa = kTapOff + 16 * (g & 1) - m - kMfmaLeft + R;
    const int pq = pa >> 2, pb = pa & 3;
    v4i a[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const uint32_t *zr = taps + (2 * s + (g >> 1)) * (kTapRow / 4) + pq;
        uint32_t z[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) z[k] = zr[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[s][k] = (int)__builtin_amdgcn_alignbyte(z[k + 1], z[k], pb);
    }
    // The band row of output column i holds each tap once: its byte sum
    // (over the four lanes of that row) is sum(weights).
    int wsum = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < 4; ++k) wsum = __builtin_amdgcn_sdot4(a[s][k], 0x01010101, wsum, false);
    wsum += __shfl_xor(wsum, 16);
    wsum += __shfl_xor(wsum, 32);
    const int bias = 128 * wsum;

    const uint8_t *lane_rows = rows + (m + (g >> 1)) * kMfmaRow + 16 * (g & 1);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(out + plane, 0, h * w, kBufferFlags);
    // This wave's 16 output rows in LDS, after the staged rows.
    uint8_t *obuf = rows + (tile_rows + 2 * R + 1) * kMfmaRow + wave * kMfmaN * kMfmaRow;
    for (int r0 = wave * rpw; r0 < (wave + 1) * rpw; r0 += kMfmaN) {
        if (y0 + r0 >= h) break;  // uniform: the wave's remaining rows are below the image
        v4i acc[kMfmaBlocks];
#pragma unroll
        for (int b = 0; b < kMfmaBlocks; ++b) acc[b] = v4i{bias, bias, bias, bias};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int b = 0; b < kMfmaBlocks; ++b) {
                const v4i bv = *(const v4i *)(lane_rows + (r0 + 2 * s) * kMfmaRow + kMfmaN * b);
                acc[b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], bv, acc[b], 0, 0, 0);
            }
        }
        // Lane (m, g) puts row m, columns 16 b + 4 g .. + 3 into the wave's LDS
        // rows; then each row's bytes leave as 16-byte stores of consecutive
        // lanes (LPR lanes per row, 64 / LPR rows per store instruction).
        // Stored straight from the MFMA layout (16 rows of 16 bytes per store
        // instruction, each row piece written by several of them) the 64-column
        // kernel took 11.5 us instead of 6.4 us at 1080p RGB, 7 x 7.
#pragma unroll
        for (int b = 0; b < kMfmaBlocks; ++b)
            *(uint32_t *)(obuf + m * kMfmaRow + kMfmaN * b + 4 * g) = pack_mfma_u8(acc[b], shift);
        constexpr int LPR = kMfmaTileW / 16, RPI = kLanes / LPR;
#pragma unroll
        for (int i = 0; i < kMfmaN / RPI; ++i) {
            const int rr = RPI * i + lane / LPR, cc = 16 * (lane % LPR);
            const v4i v = *(const v4i *)(obuf + rr * kMfmaRow + cc);
            store16_mfma_u8(rs, h, w, y0 + r0 + rr, x0 + cc, aligned != 0, v);
        }
    }
}

template <int R>
hipError_t launch_u8_mfma_t(const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h, int w, int shift,
                            int rpw, int wpg, hipStream_t s) {
    rpw = std::max(kMfmaN, (rpw + kMfmaN - 1) / kMfmaN * kMfmaN);
    const int tile_rows = rpw * wpg;
    const int lds = mfma_lds_bytes<R>(tile_rows, wpg);
    if (lds > 64 * 1024) return hipErrorInvalidValue;  // PF_U8_MFMA_TILE_MAX rows fit
    const int64_t tiles_x = cdiv(w, kMfmaTileW), tiles_y = cdiv(h, tile_rows);
    const int64_t per_plane = tiles_x * tiles_y;
    const int64_t ntiles = per_plane * c;
    if (ntiles > INT32_MAX) return hipErrorInvalidValue;
    const int aligned = (w % 4 == 0) && ((uintptr_t)in % 4 == 0) && ((uintptr_t)out % 4 == 0);
    hipLaunchKernelGGL((k_filter_u8_mfma<R>), dim3((unsigned)ntiles), dim3(wpg * kLanes), lds, s, in, filt, out, h,
                       w, shift, aligned, rpw, (int)tiles_x, (int)per_plane, (int)ntiles);
    return hipGetLastError();
}

}  // namespace dev

hipError_t launch_u8_mfma(int r, const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h, int w, int shift,
                          int rpw, int wpg, hipStream_t s) {
    switch (r) {
        case 1: return dev::launch_u8_mfma_t<1>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 2: return dev::launch_u8_mfma_t<2>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 3: return dev::launch_u8_mfma_t<3>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 4: return dev::launch_u8_mfma_t<4>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 5: return dev::launch_u8_mfma_t<5>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 6: return dev::launch_u8_mfma_t<6>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 7: return dev::launch_u8_mfma_t<7>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        case 8: return dev::launch_u8_mfma_t<8>(in, filt, out, c, h, w, shift, rpw, wpg, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pf
