/* Timing driver for the CPU baseline (test and benchmark infrastructure,
 * not part of the product): runs the oracle's own functions, unchanged, on
 * one host thread or on several with OpenMP.
 *
 * Parallel runs split an image into bands of output rows; each band calls
 * the oracle on the input rows it needs (the band plus r rows above and
 * below, clipped to the image) and keeps its own output rows. A kept row's
 * window never reaches a band cut that is not an image edge, so the result
 * is bit for bit the oracle's on the whole image (every output element is
 * an independent iteration, Sec. II-B.3). Batches run one image per task.
 * Each timing is the median of `reps` runs on CLOCK_MONOTONIC. */
#define _POSIX_C_SOURCE 199309L
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

void ref_filter2d_f32(int h, int w, int r, const float *in, const float *f, float *out);
int ref_filter_sep_f32(int h, int w, int r, const float *in, const float *fx, const float *fy, float *out);
void ref_filter2d_u8(int c, int h, int w, int r, int shift, const uint8_t *in, const int8_t *f, uint8_t *out);

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int cmp_d(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static double median(double *t, int n)
{
    qsort(t, (size_t)n, sizeof(double), cmp_d);
    return t[n / 2];
}

/* kind 0: 2D (f: (2r+1)^2 taps), 1: separable (f: fx then fy), 2: uint8
 * planes (c planes, f: int8 taps, shift). One band of output rows
 * [y0, y1) of plane p, through a scratch band buffer. */
static int run_band(int kind, int c, int h, int w, int r, int shift, const void *in, const void *f, void *out,
                    int p, int y0, int y1)
{
    const int lo = y0 - r < 0 ? 0 : y0 - r, hi = y1 + r > h ? h : y1 + r;
    const int hb = hi - lo;
    const size_t es = kind == 2 ? 1 : 4;
    const size_t plane = (size_t)h * (size_t)w;
    const char *src = (const char *)in + es * ((size_t)p * plane + (size_t)lo * (size_t)w);
    char *dst = (char *)out + es * ((size_t)p * plane + (size_t)y0 * (size_t)w);
    char *tmp = malloc(es * (size_t)hb * (size_t)w);
    if (!tmp)
        return -1;
    int rc = 0;
    if (kind == 0) {
        ref_filter2d_f32(hb, w, r, (const float *)src, (const float *)f, (float *)tmp);
    } else if (kind == 1) {
        rc = ref_filter_sep_f32(hb, w, r, (const float *)src, (const float *)f, (const float *)f + 2 * r + 1,
                                (float *)tmp);
    } else {
        ref_filter2d_u8(1, hb, w, r, shift, (const uint8_t *)src, (const int8_t *)f, (uint8_t *)tmp);
    }
    memcpy(dst, tmp + es * (size_t)(y0 - lo) * (size_t)w, es * (size_t)(y1 - y0) * (size_t)w);
    free(tmp);
    return rc;
}

/* One image (all c planes) on `threads` threads; returns the median time in
 * seconds of `reps` runs, or -1 on an allocation failure. threads = 1 calls
 * the oracle once on the whole image. */
double time_image(int kind, int c, int h, int w, int r, int shift, const void *in, const void *f, void *out,
                  int threads, int reps)
{
    double t[64];
    if (reps > 64)
        reps = 64;
    const int bands = threads * 4 < h ? threads * 4 : h;
    int fail = 0;
    for (int k = 0; k < reps; ++k) {
        const double t0 = now_s();
        if (threads <= 1) {
            if (kind == 0)
                ref_filter2d_f32(h, w, r, in, f, out);
            else if (kind == 1)
                fail |= ref_filter_sep_f32(h, w, r, in, f, (const float *)f + 2 * r + 1, out) != 0;
            else
                ref_filter2d_u8(c, h, w, r, shift, in, f, out);
        } else {
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1) reduction(| : fail)
            for (int b = 0; b < c * bands; ++b) {
                const int p = b / bands, q = b % bands;
                const int y0 = (int)((int64_t)h * q / bands), y1 = (int)((int64_t)h * (q + 1) / bands);
                if (y1 > y0)
                    fail |= run_band(kind, c, h, w, r, shift, in, f, out, p, y0, y1) != 0;
            }
        }
        t[k] = now_s() - t0;
    }
    return fail ? -1.0 : median(t, reps);
}

/* A batch of n FP32 images with separable filters (fx then fy at
 * foff[i]), one image per task; median seconds of `reps` runs. */
double time_batch_sep(int n, const int *h, const int *w, const int *r, const int64_t *off, const float *in,
                      const float *filt, const int64_t *foff, float *out, int threads, int reps)
{
    double t[64];
    if (reps > 64)
        reps = 64;
    int fail = 0;
    for (int k = 0; k < reps; ++k) {
        const double t0 = now_s();
#pragma omp parallel for num_threads(threads < 1 ? 1 : threads) schedule(dynamic, 1) reduction(| : fail)
        for (int i = 0; i < n; ++i)
            fail |= ref_filter_sep_f32(h[i], w[i], r[i], in + off[i], filt + foff[i], filt + foff[i] + 2 * r[i] + 1,
                                       out + off[i]) != 0;
        t[k] = now_s() - t0;
    }
    return fail ? -1.0 : median(t, reps);
}
