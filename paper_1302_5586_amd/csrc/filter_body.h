// HIP kernels for gfx950 (MI355X): clamp-to-edge 2D image filters.
//
// The filter is a stencil, the "regular algorithm" class the paper names
// (Sec. II), over an affine loop nest whose output iterations are
// independent (Sec. II-B.3), so every output element may be computed by any
// lane in any order. The paper's own code generation targets OpenCL through
// polyhedral tiling; these kernels are written directly for CDNA4 instead:
//
//  * A wave owns a strip of 64 lanes x 4 columns. For radii 1 and 2 every
//    lane produces 4 outputs (256 columns, 1 KiB of FP32 per row) and the
//    two outermost lanes also load the r columns beyond the strip; for
//    larger radii the outermost lane on each side (two for r > 4) only
//    loads halo columns. Horizontal neighbours come from the adjacent
//    lanes through DPP wavefront shifts (v_mov_b32_dpp wave_shr/wave_shl),
//    so the halo never passes through LDS.
//  * The wave walks down its strip (one 16-byte load per lane per row),
//    in chunks of rows that are loaded one chunk ahead of the arithmetic.
//    Each input row is folded into the 2r+1 output rows it touches, held
//    in a ring of register accumulators with compile-time slot indices, so
//    every input element is read once per tile and vertical halo rows are
//    re-read only at tile ends.
//  * Strips are loaded in one of three branch-free modes: interior (plain
//    16-byte loads), edge (the nearest in-bounds 16 bytes, each clamped
//    column picked from them) and tiny (images narrower than 4 columns).
//    Stores of edge strips and of halo lanes go through buffer resources
//    whose range check drops the out-of-image columns. Outputs are stored
//    non-temporal.
//  * Taps are accumulated per output in the definition's order (dy outer,
//    dx inner, ascending). By default each tap is one fused multiply-add;
//    the EXACT instantiation uses a separate multiply and add (this file is
//    built with -ffp-contract=off) and reproduces the sequential C program
//    bit for bit.
//  * The separable variant does the row pass on the DPP window and the
//    column pass on the register ring: the FP32 intermediate never leaves
//    registers (8 bytes of HBM traffic per pixel instead of 16).
//  * The uint8 path packs 4 taps per v_dot4c_i32_i8. Pixels are biased by
//    -128 (xor 0x80) to fit the signed operand and the bias is added back
//    exactly as 128 * sum(weights).
//  * No LDS and no barriers: waves of a workgroup are independent, so
//    every wave exits on its own.
//
// Workgroup ids are remapped so that consecutive tiles land on the same
// XCD (xcd_remap).
#pragma once

#include <algorithm>
#include <type_traits>

#include "dev_common.h"
#include "pf_internal.h"

namespace pf {
namespace dev {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int kLanes = 64;

// Word 3 of a raw buffer resource on gfx9-class parts (32-bit data format,
// no swizzle, no stride): accesses at byte offsets >= num_records are
// dropped on store and return 0 on load.
constexpr int kBufferFlags = 0x00020000;

// Outputs are written once and not read back by the kernel: stores carry
// the non-temporal hint (nt), which streams them to HBM without holding
// lines in L2 that the inputs' halo rows could use. PF_NT_LOAD puts the
// same hint on the input loads (off by default: halo rows are read twice).
#ifndef PF_NT_STORE
#define PF_NT_STORE 1
#endif
#ifndef PF_NT_LOAD
#define PF_NT_LOAD 0
#endif
constexpr int kStoreAux = PF_NT_STORE ? 2 : 0;  // cache-policy operand of buffer stores: nt

template <class T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (PF_NT_LOAD) return __builtin_nontemporal_load(p);
    else return *p;
}

template <class T>
__device__ __forceinline__ void st(T *p, T v) {
    if constexpr (PF_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// base + 4 * off as a pointer into global memory. The sum is formed as an
// integer (a descriptor may carry an absolute address with a null base), so
// the result is cast through the global address space: from a plain integer
// the compiler could not tell global from LDS and would emit flat accesses,
// whose completion waits drain every outstanding load.
template <class T>
__device__ __forceinline__ T *global_at(T *base, int64_t off) {
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(reinterpret_cast<uintptr_t>(base) + (uint64_t)off * 4u);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
// Every lambda passed here is marked always_inline: a lambda the inliner
// leaves as a call keeps the locals it captures by reference on the stack
// (scratch memory), which the persistent batch kernel must not use.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// DPP wavefront shifts: lane i receives lane i-1 (from_left) or lane i+1
// (from_right). Lanes with no source lane receive 0; they are halo lanes
// whose outputs are never stored.
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
// The same shifts with an explicit value for the lane that has no source
// lane (lane 0 for from_left, lane 63 for from_right).
__device__ __forceinline__ float from_left_or(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right_or(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ int from_left_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int from_right_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}

template <bool EXACT>
__device__ __forceinline__ float madd(float wgt, float x, float acc) {
    if constexpr (EXACT) {
        const float p = wgt * x;  // no contraction: -ffp-contract=off
        return acc + p;
    } else {
        return __builtin_fmaf(wgt, x, acc);
    }
}


// ---------------------------------------------------------------- FP32 ---

// One input row as a lane holds it: its 4 columns and, for an aligned
// strip, R halo values: lane 0 holds columns x0-R .. x0-1 (just left of the
// strip), lane 63 columns x0+256 .. x0+255+R (just right of it); the other
// lanes' halo values are loaded but unused. Lanes 0 and 63 hand them to the
// DPP shifts as the value for the lane that has no source lane.
template <int R>
struct RowF32 {
    float v[4];
    float hv[aligned_strip(R) ? R : 1];
};

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef float f3u __attribute__((ext_vector_type(3), aligned(4)));

// N consecutive floats from a 4-byte aligned address as one vector load.
template <int N>
__device__ __forceinline__ void loadn(const float *__restrict__ p, float (&o)[N]) {
    if constexpr (N == 4) {
        const f4u q = ld(reinterpret_cast<const f4u *>(p));
        o[0] = q.x, o[1] = q.y, o[2] = q.z, o[3] = q.w;
    } else if constexpr (N == 3) {
        const f3u q = *reinterpret_cast<const f3u *>(p);
        o[0] = q.x, o[1] = q.y, o[2] = q.z;
    } else if constexpr (N == 2) {
        const f2u q = *reinterpret_cast<const f2u *>(p);
        o[0] = q.x, o[1] = q.y;
    } else {
        o[0] = p[0];
    }
}

// Load modes of a strip (strip_mode); all three are branch-free.
constexpr int kFast = kStripFast, kEdge = kStripEdge, kTiny = kStripTiny;

__device__ __forceinline__ float pick4(const f4u &t, int i) {
    return i == 0 ? t.x : (i == 1 ? t.y : (i == 2 ? t.z : t.w));
}

// Load one row for a lane: the loaded values as they come from memory
// (finish_row turns them into columns xs .. xs+3 clamped to [0, w-1] and,
// for an aligned strip, the clamped halo values). The selection is left to
// the fold so that the loads of the next chunk are not waited for when
// they are issued.
template <int R, int MODE>
__device__ __forceinline__ void load_row(const float *__restrict__ row, int xs, int x0, int w, int lane,
                                         RowF32<R> &q) {
    if constexpr (MODE == kFast || MODE == kEdge) {
        const f4u t = ld(reinterpret_cast<const f4u *>(row + vec_load_col(R, MODE, xs, w)));
        q.v[0] = t.x;
        q.v[1] = t.y;
        q.v[2] = t.z;
        q.v[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) q.v[k] = row[clampi(xs + k, 0, w - 1)];
    }
    if constexpr (aligned_strip(R)) {
        const bool left = lane < kLanes / 2;
        if constexpr (MODE == kFast) {
            loadn<R>(row + halo_load_col(R, left, x0, w), q.hv);
        } else {
            const int xh = left ? x0 - R : x0 + 4 * kLanes;
#pragma unroll
            for (int j = 0; j < R; ++j) q.hv[j] = row[clampi(xh + j, 0, w - 1)];
        }
    }
}

// Where a lane sits in its strip: what finish_row needs to clamp a row.
struct LaneCtx {
    int xs, x0, w, lane;
};

// The loaded row as columns xs .. xs+3 clamped to [0, w-1] and, for an
// aligned strip, its clamped halo values. kFast: the left halo lane of the
// first strip (left of column 0) replicates column 0, and an aligned strip
// flush with the image edge takes its halo from its own edge column. kEdge:
// the lane loaded the 4 in-bounds columns nearest to its own and picks
// each clamped column from them.
template <int R, int MODE>
__device__ __forceinline__ void finish_row(RowF32<R> &q, const LaneCtx &c) {
    if constexpr (MODE == kFast) {
        if constexpr (idle_lanes(R) > 0) {
            const bool left_of_image = c.xs < 0;
            q.v[1] = left_of_image ? q.v[0] : q.v[1];
            q.v[2] = left_of_image ? q.v[0] : q.v[2];
            q.v[3] = left_of_image ? q.v[0] : q.v[3];
        }
    } else if constexpr (MODE == kEdge) {
        const int xa = vec_load_col(R, kEdge, c.xs, c.w);
        const f4u t = {q.v[0], q.v[1], q.v[2], q.v[3]};
#pragma unroll
        for (int k = 0; k < 4; ++k) q.v[k] = pick4(t, clampi(c.xs + k, 0, c.w - 1) - xa);
    }
    if constexpr (aligned_strip(R) && MODE == kFast) {
        const bool left = c.lane < kLanes / 2;
        const bool edge = left ? (c.x0 == 0) : (c.x0 + 4 * kLanes == c.w);
        const float e = left ? q.v[0] : q.v[3];
#pragma unroll
        for (int j = 0; j < R; ++j) q.hv[j] = edge ? e : q.hv[j];
    }
}

template <int R, int VAR>
struct Weights {
    static constexpr int K = 2 * R + 1;
    static constexpr bool SEP = (VAR == PF_VAR_SEPARABLE);
    float w2[SEP ? 1 : K * K];
    float fx[SEP ? K : 1];
    float fy[SEP ? K : 1];
    LaneCtx lc;  // set per strip: where this lane sits (see finish_row)

    // fa: the (2R+1)^2 taps (DIRECT) or fx (separable kinds); fb: fy.
    __device__ __forceinline__ Weights(const float *__restrict__ fa, const float *__restrict__ fb) {
        if constexpr (VAR == PF_VAR_DIRECT) {
#pragma unroll
            for (int i = 0; i < K * K; ++i) w2[i] = fa[i];
        } else if constexpr (VAR == PF_VAR_SEPARABLE) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                fx[i] = fa[i];
                fy[i] = fb[i];
            }
        } else {
            // 2D taps of a separable filter: fy[a] * fx[b] rounded once to FP32.
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int b = 0; b < K; ++b) w2[a * K + b] = fb[a] * fa[b];
        }
    }
};

// Fold one input row into the accumulator ring.
//   RES: the row's index modulo K (compile time).
//   IPRO >= 0: the row is prologue row IPRO (< 2R): skip outputs j < 0.
// Output j of the strip collects input rows j .. j+2R (dy = -R .. R) and
// lives in ring slot j mod K.
template <int R, int VAR, bool EXACT, int RES, int IPRO, int MODE>
__device__ __forceinline__ void fold_row_f32(const Weights<R, VAR> &wt, const RowF32<R> &q0,
                                             float (&acc)[2 * R + 1][4]) {
    RowF32<R> q = q0;
    finish_row<R, MODE>(q, wt.lc);
    constexpr int K = 2 * R + 1;
    constexpr int NB = halo_lanes(R);
    constexpr int C = 4 * NB;
    constexpr int NW = 4 * (2 * NB + 1);
    const float *v = q.v;
    // win[C + c] is column xs + c of this lane's row, c in [-4 NB, 4 NB + 4).
    float win[NW];
#pragma unroll
    for (int k = 0; k < 4; ++k) win[C + k] = v[k];
    if constexpr (aligned_strip(R)) {
        // Only the R columns on each side are needed; lanes 0 and 63 take
        // them from the strip's halo columns instead of a neighbour.
#pragma unroll
        for (int j = 0; j < R; ++j) {
            win[C - R + j] = from_left_or(q.hv[j], v[4 - R + j]);
            win[C + 4 + j] = from_right_or(q.hv[j], v[j]);
        }
    } else {
        float l[4] = {v[0], v[1], v[2], v[3]};
        float r[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
        for (int m = 1; m <= NB; ++m) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                l[k] = from_left(l[k]);
                r[k] = from_right(r[k]);
                win[C - 4 * m + k] = l[k];
                win[C + 4 * m + k] = r[k];
            }
        }
    }
    if constexpr (VAR == PF_VAR_SEPARABLE) {
        float t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            t[k] = 0.0f;
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) t[k] = madd<EXACT>(wt.fx[dx + R], win[C + k + dx], t[k]);
        }
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            // output j = i - R - dy; in the prologue i = IPRO and j < 0 is skipped
            if (IPRO >= 0 && IPRO - R - dy < 0) continue;
            const int slot = ((RES - R - dy) % K + K) % K;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[slot][k] = madd<EXACT>(wt.fy[dy + R], t[k], acc[slot][k]);
        }
    } else {
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            if (IPRO >= 0 && IPRO - R - dy < 0) continue;
            const int slot = ((RES - R - dy) % K + K) % K;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int dx = -R; dx <= R; ++dx)
                    acc[slot][k] = madd<EXACT>(wt.w2[(dy + R) * K + dx + R], win[C + k + dx], acc[slot][k]);
        }
    }
}

template <int R, int CHUNK>
constexpr int chunk_rows() {
    return chunk_rows_of(R, CHUNK);
}

// Load input rows [i0, i0 + CH) of a strip. Rows past the strip's last
// input row `last` repeat that row (a cache hit), so the loads of the next
// chunk are issued without a branch: a branch around them would make the
// wait counts at the join conservative and serialize the chunks.
template <int R, int CH, int MODE>
__device__ __forceinline__ void load_chunk(const float *__restrict__ in, int h, int w, int xs, int x0, int lane,
                                           int y0, int i0, int last, RowF32<R> (&v)[CH]) {
#pragma unroll
    for (int s = 0; s < CH; ++s) {
        const int yy = clampi(y0 - R + min(i0 + s, last), 0, h - 1);
        load_row<R, MODE>(in + (int64_t)yy * w, xs, x0, w, lane, v[s]);
    }
}

// Store the 4 outputs of a lane in output row y, without a branch (so the
// wait counts of the loads in flight stay exact). kFast with every lane an
// output lane: one 16-byte store. kFast with halo lanes: one 16-byte store
// through a buffer resource whose range is the row, halo lanes passing an
// offset outside it (the hardware drops such accesses). Otherwise four
// dword stores through that resource: columns at or beyond w are dropped.
template <int MODE, int IL>
__device__ __forceinline__ void store_row(float *__restrict__ out, int w, int xs, int y, bool out_lane,
                                          const float (&a)[4]) {
    float *o = out + (int64_t)y * w;
    if constexpr (MODE == kFast && IL == 0) {
        f4u t;
        t.x = a[0];
        t.y = a[1];
        t.z = a[2];
        t.w = a[3];
        st(reinterpret_cast<f4u *>(o + xs), t);
    } else if constexpr (MODE == kFast) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(o, 0, w * 4, kBufferFlags);
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        u4 t;
        t.x = __float_as_uint(a[0]);
        t.y = __float_as_uint(a[1]);
        t.z = __float_as_uint(a[2]);
        t.w = __float_as_uint(a[3]);
        __builtin_amdgcn_raw_buffer_store_b128(t, rs, out_lane ? xs * 4 : 0x7ffffff0, 0, kStoreAux);
    } else {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(o, 0, w * 4, kBufferFlags);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int off = out_lane ? (xs + k) * 4 : 0x7ffffff0;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(a[k]), rs, off, 0, kStoreAux);
        }
    }
}

// Fold input rows [i0, i0 + CH) (all present) into the ring and store the
// outputs they complete. i0 = 2R + q*CH, so row i0 + s has ring residue
// (2R + s) mod K; the output completed by row i is i - 2R.
template <int R, int VAR, bool EXACT, int CH, int MODE>
__device__ __forceinline__ void process_chunk(const Weights<R, VAR> &wt, const RowF32<R> (&v)[CH],
                                              float (&acc)[2 * R + 1][4], float *__restrict__ out, int w, int xs,
                                              int y0, int i0, bool out_lane) {
    constexpr int K = 2 * R + 1;
    static_for<0, CH>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        constexpr int RES = (2 * R + s) % K;
        fold_row_f32<R, VAR, EXACT, RES, -1, MODE>(wt, v[s], acc);
        constexpr int done = (RES + 1) % K;
        store_row<MODE, idle_lanes(R)>(out, w, xs, y0 + i0 + s - 2 * R, out_lane, acc[done]);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[done][k] = 0.0f;
    });
}

// Up to K rows from i0 (each only if below nin), loaded one by one; i0 is
// congruent to OFF modulo K. The tail of the pipelined loop, and (OFF = 0,
// from row 0) the whole row loop of the compact form for large radii.
template <int R, int VAR, bool EXACT, int OFF, int MODE>
__device__ __forceinline__ void rows_group_f32(const Weights<R, VAR> &wt, const float *__restrict__ in,
                                               float *__restrict__ out, float (&acc)[2 * R + 1][4], int h, int w,
                                               int xs, int x0, int lane, int y0, int rows, int i0, int nin,
                                               bool out_lane) {
    constexpr int K = 2 * R + 1;
    // Radii up to 4: the group's rows are all loaded first (rows past nin
    // repeat the last one and are not folded), so their loads overlap
    // instead of each being waited for before the next is issued.
    constexpr bool AHEAD = R <= 4;
    RowF32<R> va[AHEAD ? K : 1];
    if constexpr (AHEAD) {
        static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            const int yy = clampi(y0 - R + min(i0 + s, nin - 1), 0, h - 1);
            load_row<R, MODE>(in + (int64_t)yy * w, xs, x0, w, lane, va[s]);
        });
    }
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        if (i0 + s < nin) {
            constexpr int RES = (OFF + s) % K;
            RowF32<R> v;
            if constexpr (AHEAD) {
                v = va[s];
            } else {
                const int yy = clampi(y0 - R + i0 + s, 0, h - 1);
                load_row<R, MODE>(in + (int64_t)yy * w, xs, x0, w, lane, v);
            }
            fold_row_f32<R, VAR, EXACT, RES, -1, MODE>(wt, v, acc);
            const int j = i0 + s - 2 * R;
            constexpr int done = (RES + 1) % K;
            if (j >= 0 && j < rows) store_row<MODE, idle_lanes(R)>(out, w, xs, y0 + j, out_lane, acc[done]);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[done][k] = 0.0f;
        }
    });
}

// The row loop for radii 0..4: prologue rows 0..2R-1, then full chunks
// of CH rows in two alternating register sets (the loads of one chunk are
// in flight while the other is folded; no per-row branch inside the loop),
// then the remaining rows in groups of K.
template <int R, int VAR, bool EXACT, int MODE, int CHUNK>
__device__ __forceinline__ void rows_pipelined_f32(const Weights<R, VAR> &wt, const float *__restrict__ in,
                                                   float *__restrict__ out, float (&acc)[2 * R + 1][4], int h, int w,
                                                   int xs, int x0, int lane, int y0, int rows, bool out_lane) {
    constexpr int K = 2 * R + 1;
    constexpr int CH = chunk_rows<R, CHUNK>();
    const int nin = rows + 2 * R;
    int i0 = 2 * R;
    if (i0 + CH <= nin) {
        RowF32<R> pv[2 * R > 0 ? 2 * R : 1];
        if constexpr (R > 0) {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i)
                load_row<R, MODE>(in + (int64_t)clampi(y0 - R + i, 0, h - 1) * w, xs, x0, w, lane, pv[i]);
        }
        const int last = nin - 1;
        RowF32<R> va[CH], vb[CH];
        load_chunk<R, CH, MODE>(in, h, w, xs, x0, lane, y0, i0, last, va);
        if constexpr (R > 0) {
            // Prologue: input rows 0 .. 2R-1 complete no output.
            static_for<0, 2 * R>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = decltype(ic)::value;
                fold_row_f32<R, VAR, EXACT, i % K, i, MODE>(wt, pv[i], acc);
            });
        }
        for (;;) {
            load_chunk<R, CH, MODE>(in, h, w, xs, x0, lane, y0, i0 + CH, last, vb);
            process_chunk<R, VAR, EXACT, CH, MODE>(wt, va, acc, out, w, xs, y0, i0, out_lane);
            i0 += CH;
            if (i0 + CH > nin) break;
            load_chunk<R, CH, MODE>(in, h, w, xs, x0, lane, y0, i0 + CH, last, va);
            process_chunk<R, VAR, EXACT, CH, MODE>(wt, vb, acc, out, w, xs, y0, i0, out_lane);
            i0 += CH;
            if (i0 + CH > nin) break;
        }
    } else if constexpr (R > 0) {
        // Too few rows for one chunk: the prologue rows one by one.
        for (int i = 0; i < 2 * R; i += K)
            rows_group_f32<R, VAR, EXACT, 0, MODE>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, i, 2 * R, out_lane);
    }
    // Rows left after the last full chunk; i0 = 2R (mod K).
    for (; i0 < nin; i0 += K)
        rows_group_f32<R, VAR, EXACT, (2 * R) % K, MODE>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, i0, nin,
                                                          out_lane);
}

// One wave computes output rows [y0, y0 + rows) of columns [x0, x0 + strip
// width) of one image plane.
template <int R, int VAR, bool EXACT, int CHUNK = PF_CHUNK>
__device__ __forceinline__ void strip_f32(const float *__restrict__ in, const float *__restrict__ fa,
                                          const float *__restrict__ fb, float *__restrict__ out, int h, int w,
                                          int x0, int y0, int rows, int lane) {
    constexpr int K = 2 * R + 1;
    constexpr int IL = idle_lanes(R);
    Weights<R, VAR> wt(fa, fb);
    const int xs = lane_col(R, x0, lane);
    wt.lc = LaneCtx{xs, x0, w, lane};
    const bool out_lane = (lane >= IL) && (lane < kLanes - IL) && (xs < w);
    float acc[K][4];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[s][k] = 0.0f;

    if constexpr (R > 4) {
        // Compact form for large radii: one guarded copy of the K-row body
        // (the first 2R rows fold into outputs j < 0 that are never stored).
        const int nin = rows + 2 * R;
        for (int i0 = 0; i0 < nin; i0 += K)
            rows_group_f32<R, VAR, EXACT, 0, kTiny>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, i0, nin, out_lane);
    } else {
        const int mode = strip_mode(R, x0, w);
        if (mode == kFast) {
            rows_pipelined_f32<R, VAR, EXACT, kFast, CHUNK>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, out_lane);
        } else if (mode == kEdge) {
            rows_pipelined_f32<R, VAR, EXACT, kEdge, CHUNK>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, out_lane);
        } else {
            const int nin = rows + 2 * R;
            for (int i0 = 0; i0 < nin; i0 += K)
                rows_group_f32<R, VAR, EXACT, 0, kTiny>(wt, in, out, acc, h, w, xs, x0, lane, y0, rows, i0, nin,
                                                        out_lane);
        }
    }
}

// Tile number -> (strip x, strip y). Tiles are numbered row-major, so the
// waves in flight at any moment cover whole bands of consecutive image
// rows: a compact, slowly advancing window of HBM pages (and of address
// translations), which MI355X serves markedly faster than the same tiles
// taken strip by strip down the image.
// The uint8 kernel keeps column-major order (strip by strip), which
// measured faster for it.
#ifndef PF_U8_COLMAJOR
#define PF_U8_COLMAJOR 1
#endif
// Rows per pipelined uint8 chunk: a multiple of K near this many.
#ifndef PF_U8_CHUNK
#define PF_U8_CHUNK 8
#endif
template <bool COLMAJOR = kTileColMajorF32>
__device__ __forceinline__ void tile_xy(int t, int strips_x, int strips_y, int &sx, int &sy) {
    tile_strip(COLMAJOR, t, strips_x, strips_y, sx, sy);
}

// Single-image kernel: one wave tile per task.
template <int R, int VAR, bool EXACT>
__global__ __launch_bounds__(512) void k_filter_f32(const float *__restrict__ in, const float *__restrict__ fa,
                                                    const float *__restrict__ fb, float *__restrict__ out, int h,
                                                    int w, int by, int strips_x, int strips_y, int ntasks) {
    const int wpg = blockDim.x / kLanes;
    const int wave = uniform(threadIdx.x / kLanes);
    const int lane = threadIdx.x % kLanes;
    const int t = xcd_remap(blockIdx.x, gridDim.x) * wpg + wave;
    if (t >= ntasks) return;
    int sx, sy;
    tile_xy(t, strips_x, strips_y, sx, sy);
    const int y0 = sy * by;
    strip_f32<R, VAR, EXACT>(in, fa, fb, out, h, w, sx * strip_width(R), y0, min(by, h - y0), lane);
}

// Persistent batch kernel: a fixed grid of workgroups walks the list of all
// images' wave tiles with a static stride (tiles in image order, row-major
// inside each image). Each entry names an image and a tile; the image
// descriptor gives the radius, variant, tile height and arena offsets.
template <int RLO, int RHI, bool EXACT, int VMASK>
__global__ __launch_bounds__(512) void k_batch_f32(const BatchImg *__restrict__ imgs,
                                                   const BatchTask *__restrict__ tasks, int ntasks,
                                                   const float *__restrict__ in, const float *__restrict__ filt,
                                                   float *__restrict__ out) {
    const int wpg = blockDim.x / kLanes;
    const int wave = uniform(threadIdx.x / kLanes);
    const int lane = threadIdx.x % kLanes;
    const int stride = gridDim.x * wpg;
    for (int t = xcd_remap(blockIdx.x, gridDim.x) * wpg + wave; t < ntasks; t += stride) {
        const BatchTask tk = tasks[t];
        const BatchImg d = imgs[uniform(tk.img)];
        int sx, sy;
        tile_xy(uniform(tk.tile), d.strips_x, d.strips_y, sx, sy);
        const int y0 = sy * d.by;
        const int rows = min(d.by, d.h - y0);
        const float *src = global_at(in, d.in_off);
        float *dst = global_at(out, d.out_off);
        const float *fa = global_at(filt, d.filt_off);
        const float *fb = fa + 2 * d.r + 1;
        // Only the variants in VMASK are compiled in: the register budget of
        // the kernel is the largest of its bodies.
        static_for<RLO, RHI + 1>([&](auto rc) __attribute__((always_inline)) {
            constexpr int RR = decltype(rc)::value;
            if (d.r == RR) {
                static_for<0, 3>([&](auto vc) __attribute__((always_inline)) {
                    constexpr int VV = decltype(vc)::value;
                    if constexpr ((VMASK >> VV) & 1) {
                        if (d.var == VV)
                            strip_f32<RR, VV, EXACT, PF_BATCH_CHUNK>(src, fa, fb, dst, d.h, d.w, sx * strip_width(RR), y0,
                                                            rows, lane);
                    }
                });
            }
        });
    }
}

// --------------------------------------------------------------- uint8 ---

constexpr int floordiv4(int u) { return u >= 0 ? u / 4 : -((-u + 3) / 4); }

template <int R>
struct WeightsU8 {
    static constexpr int K = 2 * R + 1;
    static constexpr int ND = (K + 3) / 4;  // dwords per filter row
    static constexpr int PAD = 4 * ND - K;  // zero taps in front of each row
    int32_t wd[K][ND];
    int32_t bias;  // 128 * sum of weights
    // Byte selector (v_perm_b32) that turns the dword a lane loads into its
    // 4 clamped pixels; set per strip (see load_u8). Applied where a row is
    // folded, not where it is loaded, so that the load of the next chunk is
    // not waited for early.
    uint32_t sel = 0x03020100u;

    __device__ __forceinline__ explicit WeightsU8(const int8_t *__restrict__ filt) {
        int s = 0;
#pragma unroll
        for (int dy = 0; dy < K; ++dy) {
#pragma unroll
            for (int m = 0; m < ND; ++m) {
                uint32_t pk = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int t = 4 * m + b - PAD;
                    if (t >= 0 && t < K) {
                        const int8_t q = filt[dy * K + t];
                        s += q;
                        pk |= (uint32_t)(uint8_t)q << (8 * b);
                    }
                }
                wd[dy][m] = (int32_t)pk;
            }
        }
        bias = 128 * s;
    }
};

// The dword a lane loads for bytes xs .. xs+3 of a row; the byte selector
// of load_sel_u8 turns it into those bytes clamped to [0, w-1], packed
// little-endian. kFast (rows 4-byte aligned, every lane's bytes end inside
// the row): the dword at xs (at 0 for the halo lane left of byte 0, which
// replicates byte 0). kEdge (aligned rows, w >= 4): the nearest in-bounds
// dword. kTiny (unaligned rows or w < 4): one clamped byte load per byte,
// already in place.
template <int MODE>
__device__ __forceinline__ uint32_t load_u8(const uint8_t *__restrict__ row, int xs, int w) {
    if constexpr (MODE == kFast) {
        return ld(reinterpret_cast<const uint32_t *>(row + max(xs, 0)));
    } else if constexpr (MODE == kEdge) {
        return ld(reinterpret_cast<const uint32_t *>(row + clampi(xs, 0, w - 4)));
    } else {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) v |= (uint32_t)row[clampi(xs + k, 0, w - 1)] << (8 * k);
        return v;
    }
}

// Byte selector for load_u8's dword in mode MODE (v_perm_b32 byte k = the
// index, within that dword, of clamped byte xs + k).
template <int MODE>
__device__ __forceinline__ uint32_t load_sel_u8(int xs, int w) {
    if constexpr (MODE == kFast) {
        return xs < 0 ? 0u : 0x03020100u;
    } else if constexpr (MODE == kEdge) {
        const int xa = clampi(xs, 0, w - 4);
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) s |= (uint32_t)(clampi(xs + k, 0, w - 1) - xa) << (8 * k);
        return s;
    } else {
        return 0x03020100u;
    }
}

template <int R, int RES, int IPRO>
__device__ __forceinline__ void fold_row_u8(const WeightsU8<R> &wt, uint32_t own, int (&acc)[2 * R + 1][4]) {
    constexpr int K = 2 * R + 1;
    constexpr int NB = halo_lanes(R);
    constexpr int ND = WeightsU8<R>::ND;
    constexpr int PAD = WeightsU8<R>::PAD;
    uint32_t win[2 * NB + 1];
    win[NB] = __builtin_amdgcn_perm(own, own, wt.sel) ^ 0x80808080u;  // p - 128 as signed bytes
    {
        int l = (int)win[NB], r = (int)win[NB];
#pragma unroll
        for (int m = 1; m <= NB; ++m) {
            l = from_left_i(l);
            r = from_right_i(r);
            win[NB - m] = (uint32_t)l;
            win[NB + m] = (uint32_t)r;
        }
    }
    // D[k][m]: the 4 bytes multiplied by filter dword m for output column k.
    int32_t D[4][ND];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int m = 0; m < ND; ++m) {
            const int u0 = k - R - PAD + 4 * m + 4 * NB;  // window byte of the dword's first byte
            const int lo = floordiv4(u0);
            const int sh = u0 - 4 * lo;
            const uint32_t a = (lo >= 0 && lo <= 2 * NB) ? win[lo >= 0 && lo <= 2 * NB ? lo : 0] : 0u;
            const uint32_t b = (lo + 1 >= 0 && lo + 1 <= 2 * NB) ? win[lo + 1 >= 0 && lo + 1 <= 2 * NB ? lo + 1 : 0] : 0u;
            D[k][m] = (int32_t)(sh == 0 ? a : __builtin_amdgcn_alignbyte(b, a, sh));
        }
    }
    // The row's tap dy = -R is the first term of output slot RES: that
    // accumulator starts from the bias (128 * sum of weights, undoing the
    // -128 on every pixel) instead of from a zeroed register.
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        if (IPRO >= 0 && IPRO - R - dy < 0) continue;
        const int slot = ((RES - R - dy) % K + K) % K;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int m = 0; m < ND; ++m) {
                const int prev = (dy == -R && m == 0) ? wt.bias : acc[slot][k];
                acc[slot][k] = __builtin_amdgcn_sdot4(D[k][m], wt.wd[dy + R][m], prev, false);
            }
    }
}

// Finish 4 outputs (arithmetic shift, saturate; the bias is already in
// the sums) and store them through a buffer resource spanning the row: one
// dword store in kFast, else four byte stores; bytes at or beyond w and
// halo lanes (offset outside the range) are dropped by the hardware. No
// branch.
template <int MODE>
__device__ __forceinline__ void store_u8(uint8_t *__restrict__ row, int xs, int w, bool out_lane, const int (&a)[4],
                                         int shift) {
    uint32_t pk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int q = clampi(a[k] >> shift, 0, 255);  // arithmetic shift of a signed int
        // Keep each saturated byte opaque until it is packed: fused into the
        // gfx950 packed shift-and-saturate instruction, the pair of bytes
        // came back with the upper half of the dword not cleared, and the
        // OR with bytes 2 and 3 then set them to 255.
        asm volatile("" : "+v"(q));
        pk |= (uint32_t)q << (8 * k);
    }
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, w, kBufferFlags);
    if constexpr (MODE == kFast) {
        __builtin_amdgcn_raw_buffer_store_b32(pk, rs, out_lane ? xs : 0x7ffffff0, 0, kStoreAux);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(pk >> (8 * k)), rs, out_lane ? xs + k : 0x7ffffff0, 0, kStoreAux);
    }
}

template <int R, int CH, int MODE>
__device__ __forceinline__ void load_chunk_u8(const uint8_t *__restrict__ in, int h, int w, int xs, int y0, int i0,
                                              int last, uint32_t (&v)[CH]) {
#pragma unroll
    for (int s = 0; s < CH; ++s) v[s] = load_u8<MODE>(in + (int64_t)clampi(y0 - R + min(i0 + s, last), 0, h - 1) * w, xs, w);
}

// Fold rows [i0, i0 + CH) (all present; i0 = 2R + q*CH) and store the
// outputs they complete.
template <int R, int CH, int MODE>
__device__ __forceinline__ void process_chunk_u8(const WeightsU8<R> &wt, const uint32_t (&v)[CH],
                                                 int (&acc)[2 * R + 1][4], uint8_t *__restrict__ out, int w,
                                                 int shift, int xs, int y0, int i0, bool out_lane) {
    constexpr int K = 2 * R + 1;
    static_for<0, CH>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        constexpr int RES = (2 * R + s) % K;
        fold_row_u8<R, RES, -1>(wt, v[s], acc);
        constexpr int done = (RES + 1) % K;
        store_u8<MODE>(out + (int64_t)(y0 + i0 + s - 2 * R) * w, xs, w, out_lane, acc[done], shift);
    });
}

// Up to K rows from i0 (those below nin), loaded one by one; i0 = OFF
// (mod K).
template <int R, int OFF, int MODE>
__device__ __forceinline__ void rows_group_u8(const WeightsU8<R> &wt, const uint8_t *__restrict__ in,
                                              uint8_t *__restrict__ out, int (&acc)[2 * R + 1][4], int h, int w,
                                              int shift, int xs, int y0, int rows, int i0, int nin, bool out_lane) {
    constexpr int K = 2 * R + 1;
    // Radii up to 4: all the group's rows are loaded first (as in
    // rows_group_f32).
    constexpr bool AHEAD = R <= 4;
    uint32_t va[AHEAD ? K : 1];
    if constexpr (AHEAD) {
#pragma unroll
        for (int s = 0; s < K; ++s)
            va[s] = load_u8<MODE>(in + (int64_t)clampi(y0 - R + min(i0 + s, nin - 1), 0, h - 1) * w, xs, w);
    }
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        if (i0 + s < nin) {
            constexpr int RES = (OFF + s) % K;
            const uint32_t v =
                AHEAD ? va[AHEAD ? s : 0] : load_u8<MODE>(in + (int64_t)clampi(y0 - R + i0 + s, 0, h - 1) * w, xs, w);
            fold_row_u8<R, RES, -1>(wt, v, acc);
            const int j = i0 + s - 2 * R;
            constexpr int done = (RES + 1) % K;
            if (j >= 0 && j < rows) store_u8<MODE>(out + (int64_t)(y0 + j) * w, xs, w, out_lane, acc[done], shift);
        }
    });
}

// The uint8 row loop: prologue, full chunks in two alternating register
// sets, then the remaining rows in groups of K (as the FP32 strip).
template <int R, int MODE>
__device__ __forceinline__ void rows_u8(const WeightsU8<R> &wt, const uint8_t *__restrict__ in,
                                        uint8_t *__restrict__ out, int (&acc)[2 * R + 1][4], int h, int w, int shift,
                                        int xs, int y0, int rows, bool out_lane) {
    constexpr int K = 2 * R + 1;
    constexpr int CH = K * (PF_U8_CHUNK / K > 0 ? PF_U8_CHUNK / K : 1);
    const int nin = rows + 2 * R;
    int i0 = 2 * R;
    if (i0 + CH <= nin) {
        const int last = nin - 1;
        uint32_t pv[2 * R > 0 ? 2 * R : 1];
        if constexpr (R > 0) {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) pv[i] = load_u8<MODE>(in + (int64_t)clampi(y0 - R + i, 0, h - 1) * w, xs, w);
        }
        uint32_t va[CH], vb[CH];
        load_chunk_u8<R, CH, MODE>(in, h, w, xs, y0, i0, last, va);
        if constexpr (R > 0) {
            static_for<0, 2 * R>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = decltype(ic)::value;
                fold_row_u8<R, i % K, i>(wt, pv[i], acc);
            });
        }
        for (;;) {
            load_chunk_u8<R, CH, MODE>(in, h, w, xs, y0, i0 + CH, last, vb);
            process_chunk_u8<R, CH, MODE>(wt, va, acc, out, w, shift, xs, y0, i0, out_lane);
            i0 += CH;
            if (i0 + CH > nin) break;
            load_chunk_u8<R, CH, MODE>(in, h, w, xs, y0, i0 + CH, last, va);
            process_chunk_u8<R, CH, MODE>(wt, vb, acc, out, w, shift, xs, y0, i0, out_lane);
            i0 += CH;
            if (i0 + CH > nin) break;
        }
    } else if constexpr (R > 0) {
        for (int i = 0; i < 2 * R; i += K)
            rows_group_u8<R, 0, MODE>(wt, in, out, acc, h, w, shift, xs, y0, rows, i, 2 * R, out_lane);
    }
    for (; i0 < nin; i0 += K)
        rows_group_u8<R, (2 * R) % K, MODE>(wt, in, out, acc, h, w, shift, xs, y0, rows, i0, nin, out_lane);
}

// The uint8 strip walk: the row ring of the FP32 strip, 4 bytes per lane,
// halo lanes on each side.
template <int R>
__device__ __forceinline__ void strip_u8(const uint8_t *__restrict__ in, const int8_t *__restrict__ filt,
                                         uint8_t *__restrict__ out, int h, int w, int shift, bool aligned,
                                         int x0, int y0, int rows, int lane) {
    constexpr int K = 2 * R + 1;
    constexpr int NB = halo_lanes(R);
    WeightsU8<R> wt(filt);
    const int xs = x0 + 4 * (lane - NB);
    const bool out_lane = (lane >= NB) && (lane < kLanes - NB) && (xs < w);
    int acc[K][4];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[s][k] = 0;
    if (aligned && x0 + 4 * (kLanes - NB) <= w) {
        wt.sel = load_sel_u8<kFast>(xs, w);
        rows_u8<R, kFast>(wt, in, out, acc, h, w, shift, xs, y0, rows, out_lane);
    } else if (aligned && w >= 4) {
        wt.sel = load_sel_u8<kEdge>(xs, w);
        rows_u8<R, kEdge>(wt, in, out, acc, h, w, shift, xs, y0, rows, out_lane);
    } else {
        wt.sel = load_sel_u8<kTiny>(xs, w);
        rows_u8<R, kTiny>(wt, in, out, acc, h, w, shift, xs, y0, rows, out_lane);
    }
}

// Wave tile (sx, sy) of a plane covers rows [sy h / strips_y, (sy+1) h /
// strips_y): the rows are spread evenly over the tiles of a strip column.
template <int R>
__global__ __launch_bounds__(512) void k_filter_u8(const uint8_t *__restrict__ in, const int8_t *__restrict__ filt,
                                                   uint8_t *__restrict__ out, int h, int w, int shift, int aligned,
                                                   int strips_x, int strips_y, int tasks_per_plane, int ntasks) {
    const int wpg = blockDim.x / kLanes;
    const int wave = uniform(threadIdx.x / kLanes);
    const int lane = threadIdx.x % kLanes;
    const int t = xcd_remap(blockIdx.x, gridDim.x) * wpg + wave;
    if (t >= ntasks) return;
    const int p = t / tasks_per_plane;
    const int local = t - p * tasks_per_plane;
    int sx, sy;
    tile_xy<PF_U8_COLMAJOR != 0>(local, strips_x, strips_y, sx, sy);
    const int y0 = (int)((int64_t)sy * h / strips_y);
    const int y1 = (int)((int64_t)(sy + 1) * h / strips_y);
    const int64_t plane = (int64_t)p * h * w;
    strip_u8<R>(in + plane, filt, out + plane, h, w, shift, aligned != 0, sx * strip_width_u8(R), y0, y1 - y0, lane);
}

}  // namespace dev
}  // namespace pf


// ------------------------------------------------------------ launchers ---
namespace pf {
namespace dev {

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <int R, int VAR, bool EXACT>
hipError_t launch_f32_t(const float *in, const float *fa, const float *fb, float *out, int h, int w, int by, int wpg,
                        hipStream_t s) {
    const int sw = strip_width(R);
    const int strips_x = cdiv(w, sw), strips_y = cdiv(h, by);
    const int64_t ntasks64 = (int64_t)strips_x * strips_y;
    if (ntasks64 > INT32_MAX) return hipErrorInvalidValue;
    const int ntasks = (int)ntasks64;
    const int grid = cdiv(ntasks, wpg);
    hipLaunchKernelGGL((k_filter_f32<R, VAR, EXACT>), dim3(grid), dim3(wpg * kLanes), 0, s, in, fa, fb, out, h, w,
                       by, strips_x, strips_y, ntasks);
    return hipGetLastError();
}

template <int R, bool EXACT>
hipError_t launch_f32_v(int var, const float *in, const float *fa, const float *fb, float *out, int h, int w, int by,
                        int wpg, hipStream_t s) {
    switch (var) {
        case PF_VAR_DIRECT:
            return launch_f32_t<R, PF_VAR_DIRECT, EXACT>(in, fa, fb, out, h, w, by, wpg, s);
        case PF_VAR_SEPARABLE:
            return launch_f32_t<R, PF_VAR_SEPARABLE, EXACT>(in, fa, fb, out, h, w, by, wpg, s);
        case PF_VAR_SEP_DIRECT:
            // Not built above PF_SEP_DIRECT_R_MAX (its taps would spill).
            if constexpr (R <= PF_SEP_DIRECT_R_MAX)
                return launch_f32_t<R, PF_VAR_SEP_DIRECT, EXACT>(in, fa, fb, out, h, w, by, wpg, s);
            else
                return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t launch_u8_t(const uint8_t *in, const int8_t *filt, uint8_t *out, int c, int h, int w, int shift, int by,
                       int wpg, hipStream_t s) {
    const int sw = strip_width_u8(R);
    const int strips_x = cdiv(w, sw);
    // The uint8 kernel is ALU-bound: its time is the number of rounds of
    // waves a SIMD runs times the rows a wave folds. Keep the rounds that
    // `by` asks for, but cut each strip column into as many tiles as fill
    // those rounds (rows spread evenly, never more than `by` per tile), so
    // the last round is not left partly idle.
    const int64_t cols = (int64_t)strips_x * c;
    const int64_t simds = 4 * (int64_t)std::max(dev_info().cus, 1);
    const int64_t asked = cdiv(h, by);
    const int64_t rounds = (cols * asked + simds - 1) / simds;
    const int64_t strips_y = std::min<int64_t>(h, std::max<int64_t>(asked, rounds * simds / cols));
    const int64_t per_plane = (int64_t)strips_x * strips_y;
    const int64_t ntasks64 = per_plane * c;
    if (ntasks64 > INT32_MAX) return hipErrorInvalidValue;
    const int ntasks = (int)ntasks64;
    const int grid = cdiv(ntasks, wpg);
    const int aligned = (w % 4 == 0) && ((uintptr_t)in % 4 == 0) && ((uintptr_t)out % 4 == 0);
    hipLaunchKernelGGL((k_filter_u8<R>), dim3(grid), dim3(wpg * kLanes), 0, s, in, filt, out, h, w, shift, aligned,
                       strips_x, (int)strips_y, (int)per_plane, ntasks);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace pf
