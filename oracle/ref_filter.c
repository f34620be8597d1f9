/*
 * Oracle for the clamp-to-edge 2D image filter.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code, header, table or
 * helper with the device path.
 *
 * What it computes is the plain definition of the filter, written as
 * sequential C99 loops: the paper fixes sequential semantics for the
 * intermediate language and requires that an ordinary C compiler can build
 * it (Sec. II, overview; Sec. II-A, design). Each output element is one
 * iteration of an affine loop nest whose iterations are independent
 * (Sec. II-B.3, the `independent` directive; Sec. III-B, vector
 * construction as a recoverably parallel map), so the loop order over
 * output elements does not change any result.
 *
 * Calling convention, following the paper's coding rules (Sec. II-B.1):
 * sizes first, then arrays declared as C99 VLAs qualified
 * `restrict const static`, no pointer arithmetic on parameters, no
 * recursion, no goto. Distinct array parameters never overlap.
 *
 * Arithmetic:
 *  - FP32 paths: start at +0.0f, taps visited with dy outer and dx inner,
 *    both ascending; each tap is an FP32 multiply rounded to nearest, then
 *    an FP32 add rounded to nearest. Build with -ffp-contract=off and
 *    without -ffast-math so that no fused multiply-add is formed.
 *  - Integer path: int32 products and sums (exact for the radii used),
 *    arithmetic right shift, saturation to [0, 255].
 *
 * The filter is a correlation (no kernel flip): tap (dy, dx) multiplies
 * in[clamp(y+dy)][clamp(x+dx)], stored at f[(dy+r)*(2r+1) + (dx+r)].
 * Clamp-to-edge replicates the border pixel along each axis.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fPIC -shared
 */
#include <stdint.h>
#include <stdlib.h>

static int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* FP32 full 2D correlation with clamp-to-edge borders, one plane. */
void ref_filter2d_f32(int h, int w, int r,
                      const float in[restrict const static h * w],
                      const float f[restrict const static (2 * r + 1) * (2 * r + 1)],
                      float out[restrict const static h * w])
{
    const int k = 2 * r + 1;
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            float acc = 0.0f;
            for (int dy = -r; dy <= r; dy++) {
                const int yy = clampi(y + dy, 0, h - 1);
                for (int dx = -r; dx <= r; dx++) {
                    const int xx = clampi(x + dx, 0, w - 1);
                    const float prod = f[(dy + r) * k + (dx + r)] * in[yy * w + xx];
                    acc = acc + prod;
                }
            }
            out[y * w + x] = acc;
        }
    }
}

/* One output element of the 2D filter, for traversal-order checks and for
 * sampled checks of large images. */
float ref_filter2d_f32_at(int h, int w, int r,
                          const float in[restrict const static h * w],
                          const float f[restrict const static (2 * r + 1) * (2 * r + 1)],
                          int y, int x)
{
    const int k = 2 * r + 1;
    float acc = 0.0f;
    for (int dy = -r; dy <= r; dy++) {
        const int yy = clampi(y + dy, 0, h - 1);
        for (int dx = -r; dx <= r; dx++) {
            const int xx = clampi(x + dx, 0, w - 1);
            const float prod = f[(dy + r) * k + (dx + r)] * in[yy * w + xx];
            acc = acc + prod;
        }
    }
    return acc;
}

/* The 2D filter with the output elements visited in a caller-given order:
 * order[i] is the linear index y*w + x of the i-th element to compute.
 * Because iterations are independent, every permutation must give the
 * same bytes as ref_filter2d_f32. */
void ref_filter2d_f32_permuted(int h, int w, int r,
                               const float in[restrict const static h * w],
                               const float f[restrict const static (2 * r + 1) * (2 * r + 1)],
                               const int64_t order[restrict const static h * w],
                               float out[restrict const static h * w])
{
    for (int64_t i = 0; i < (int64_t)h * w; i++) {
        const int y = (int)(order[i] / w);
        const int x = (int)(order[i] % w);
        out[order[i]] = ref_filter2d_f32_at(h, w, r, in, f, y, x);
    }
}

/* FP32 separable filter: the row pass (1 x (2r+1), weights fx) is
 * materialised in an FP32 temporary, then the column pass ((2r+1) x 1,
 * weights fy) reads the temporary with clamped rows. Returns 0, or -1 if
 * the temporary cannot be allocated. */
int ref_filter_sep_f32(int h, int w, int r,
                       const float in[restrict const static h * w],
                       const float fx[restrict const static 2 * r + 1],
                       const float fy[restrict const static 2 * r + 1],
                       float out[restrict const static h * w])
{
    float *tmp = (float *)malloc(sizeof(float) * (size_t)h * (size_t)w);
    if (tmp == NULL)
        return -1;
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            float acc = 0.0f;
            for (int dx = -r; dx <= r; dx++) {
                const int xx = clampi(x + dx, 0, w - 1);
                const float prod = fx[dx + r] * in[y * w + xx];
                acc = acc + prod;
            }
            tmp[y * w + x] = acc;
        }
    }
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            float acc = 0.0f;
            for (int dy = -r; dy <= r; dy++) {
                const int yy = clampi(y + dy, 0, h - 1);
                const float prod = fy[dy + r] * tmp[yy * w + x];
                acc = acc + prod;
            }
            out[y * w + x] = acc;
        }
    }
    free(tmp);
    return 0;
}

/* Integer filter on c planar uint8 planes: int32 accumulate of int8 weight
 * times uint8 pixel, arithmetic right shift by `shift`, saturate to uint8.
 * The same weights apply to every plane; planes are independent. */
void ref_filter2d_u8(int c, int h, int w, int r, int shift,
                     const uint8_t in[restrict const static c * h * w],
                     const int8_t f[restrict const static (2 * r + 1) * (2 * r + 1)],
                     uint8_t out[restrict const static c * h * w])
{
    const int k = 2 * r + 1;
    for (int p = 0; p < c; p++) {
        for (int y = 0; y < h; y++) {
            for (int x = 0; x < w; x++) {
                int32_t acc = 0;
                for (int dy = -r; dy <= r; dy++) {
                    const int yy = clampi(y + dy, 0, h - 1);
                    for (int dx = -r; dx <= r; dx++) {
                        const int xx = clampi(x + dx, 0, w - 1);
                        acc += (int32_t)f[(dy + r) * k + (dx + r)]
                             * (int32_t)in[((int64_t)p * h + yy) * w + xx];
                    }
                }
                /* Arithmetic shift written as floor division so that the
                 * result does not rest on implementation-defined >> of a
                 * negative int. */
                int32_t q;
                if (acc >= 0)
                    q = acc >> shift;
                else
                    q = -(int32_t)(((-(int64_t)acc) + ((int64_t)1 << shift) - 1) >> shift);
                out[((int64_t)p * h + y) * w + x] = (uint8_t)(q < 0 ? 0 : (q > 255 ? 255 : q));
            }
        }
    }
}
