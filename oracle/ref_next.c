/*
 * Oracle for the extensions around the clamp-to-edge filter.
 *
 * TEST INFRASTRUCTURE ONLY, like ref_filter.c: only tests, the smoke check
 * and the CPU-baseline leg of the benchmark use it; the device path shares
 * no code with it.
 *
 *  - Other border rules and chains of filter passes. The paper names image
 *    processing and fluid dynamics as accelerator DSL domains (Sec. I),
 *    stencils as a regular algorithm class (Sec. II), and cross-component
 *    optimisation that pools several kernels' dependence information
 *    (Sec. II). A chain of passes is that composition, computed here one
 *    whole pass at a time.
 *  - Reductions: the `reduction` directive (Sec. II-B.3) and OptiML's `sum`
 *    mapped to a for loop with a reduction (Sec. III-B); the histogram is
 *    the indirect increment A[t[i]]++ of the `independent` example
 *    (Sec. II-B.3) with repeated indices, i.e. a reduction per bin.
 *  - OP2's edge-to-cell increment (Sec. III-A): the par_loop is the plain
 *    for loop over edges that calls the kernel on (array, index) pairs.
 *
 * Same arithmetic rules as ref_filter.c: FP32 multiply then FP32 add,
 * taps with dy outer and dx inner ascending, no fused multiply-add
 * (build with -ffp-contract=off).
 */
#include <stdint.h>
#include <stdlib.h>

enum { BORDER_CLAMP = 0, BORDER_ZERO = 1, BORDER_REFLECT = 2, BORDER_MIRROR = 3 };

/* Map an index that may lie outside [0, n) to the source index of the
 * border rule; returns -1 where the rule reads a zero. */
static int border_index(int i, int n, int border)
{
    if (i >= 0 && i < n)
        return i;
    switch (border) {
    case BORDER_CLAMP:
        return i < 0 ? 0 : n - 1;
    case BORDER_ZERO:
        return -1;
    case BORDER_REFLECT: {          /* period 2n: a b c d | d c b a */
        const int p = 2 * n;
        int m = i % p;
        if (m < 0)
            m += p;
        return m < n ? m : p - 1 - m;
    }
    case BORDER_MIRROR: {           /* period 2n-2: a b c d | c b */
        if (n == 1)
            return 0;
        const int p = 2 * n - 2;
        int m = i % p;
        if (m < 0)
            m += p;
        return m < n ? m : p - m;
    }
    default:
        return -2;
    }
}

/* FP32 2D correlation with a chosen border rule. Returns 0, or -1 for an
 * unknown border rule. */
int ref_filter2d_f32_border(int h, int w, int r, int border,
                            const float in[restrict const static h * w],
                            const float f[restrict const static (2 * r + 1) * (2 * r + 1)],
                            float out[restrict const static h * w])
{
    if (border < BORDER_CLAMP || border > BORDER_MIRROR)
        return -1;
    const int k = 2 * r + 1;
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            float acc = 0.0f;
            for (int dy = -r; dy <= r; dy++) {
                const int yy = border_index(y + dy, h, border);
                for (int dx = -r; dx <= r; dx++) {
                    const int xx = border_index(x + dx, w, border);
                    const float v = (yy < 0 || xx < 0) ? 0.0f : in[yy * w + xx];
                    const float prod = f[(dy + r) * k + (dx + r)] * v;
                    acc = acc + prod;
                }
            }
            out[y * w + x] = acc;
        }
    }
    return 0;
}

/* `passes` applications of the 2D filter; pass p reads the FP32 output of
 * pass p-1. Returns 0, or -1 for bad arguments or a failed allocation. */
int ref_filter_chain_f32(int h, int w, int r, int passes, int border,
                         const float in[restrict const static h * w],
                         const float f[restrict const static (2 * r + 1) * (2 * r + 1)],
                         float out[restrict const static h * w])
{
    if (passes < 1)
        return -1;
    float *a = (float *)malloc(sizeof(float) * (size_t)h * (size_t)w);
    float *b = (float *)malloc(sizeof(float) * (size_t)h * (size_t)w);
    if (a == NULL || b == NULL) {
        free(a);
        free(b);
        return -1;
    }
    for (int64_t i = 0; i < (int64_t)h * w; i++)
        a[i] = in[i];
    int rc = 0;
    for (int p = 0; p < passes && rc == 0; p++) {
        float *dst = (p == passes - 1) ? out : b;
        rc = ref_filter2d_f32_border(h, w, r, border, a, f, dst);
        if (p != passes - 1) {
            float *t = a;
            a = b;
            b = t;
        }
    }
    free(a);
    free(b);
    return rc;
}

/* Sum of n FP32 values, accumulated in float64 in index order. */
double ref_sum_f32(int64_t n, const float x[restrict const static n])
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; i++)
        acc = acc + (double)x[i];
    return acc;
}

/* hist[v] = number of i with x[i] == v, for v in 0..255. */
void ref_hist256_u8(int64_t n, const uint8_t x[restrict const static n],
                    int64_t hist[restrict const static 256])
{
    for (int v = 0; v < 256; v++)
        hist[v] = 0;
    for (int64_t i = 0; i < n; i++)
        hist[x[i]] += 1;
}

/* OP2 edge-to-cell increment: each edge adds its value to both cells it
 * touches, edges visited in index order. */
void ref_edge_inc_f64(int ncells, int nedges,
                      const int32_t edge_to_cells[restrict const static 2 * nedges],
                      const double edge[restrict const static nedges],
                      double cell[restrict const static ncells])
{
    for (int i = 0; i < nedges; i++) {
        cell[edge_to_cells[2 * i + 1]] += edge[i];
        cell[edge_to_cells[2 * i]] += edge[i];
    }
}
