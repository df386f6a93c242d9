/*
 * CPU oracle for direct 2D image convolution — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library. The product path (the HIP library) never calls it and
 * shares no code with it.
 *
 * What it computes. The paper's first benchmark kernel is the BAT-suite 2D
 * convolution (Section 5, "Benchmark kernels"; its tunable parameters are in
 * Table 1, its results in Tables 3 and 4). The paper names the kernel but does
 * not print its formula; the definition used here is the plain "valid"
 * cross-correlation that the kernel computes, with no filter flip and no
 * implicit padding (the input already carries the halo):
 *
 *   out[y][x] = sum_{i<fh} sum_{j<fw} in[y+i][x+j] * f[i][j]
 *   S[y][x]   = sum_{i<fh} sum_{j<fw} |in[y+i][x+j]| * |f[i][j]|
 *
 * for 0 <= y < H, 0 <= x < W, with the input (H+fh-1) x (W+fw-1) and the
 * filter fh x fw, all row-major FP32. Both sums are formed in FP64, in the
 * order written (i ascending, then j ascending). The product of two FP32
 * values is exact in FP64, so each term is exact; only the FP64 additions
 * round. S is the denominator of the per-point normalised error used by the
 * parity tests.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math, no contraction).
 */
#include <math.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int bad_shape(long out_h, long out_w, long fh, long fw)
{
    return out_h < 0 || out_w < 0 || fh < 1 || fw < 1;
}

/* One output point: the double sum of the definition above. */
static void one_point(const float *in, const float *f, long pitch, long fh, long fw,
                      long y, long x, double *value, double *abs_sum)
{
    double s = 0.0, a = 0.0;
    for (long i = 0; i < fh; ++i) {
        const float *row = in + (y + i) * pitch + x;
        const float *frow = f + i * fw;
        for (long j = 0; j < fw; ++j) {
            double v = (double)row[j];
            double w = (double)frow[j];
            s += v * w;
            a += fabs(v) * fabs(w);
        }
    }
    *value = s;
    *abs_sum = a;
}

/* Every output point. out and abs_sum (may be NULL) are H*W doubles.
 * Returns 0, or -1 on an invalid shape or a NULL required pointer. */
int oracle_conv2d_f64(const float *in, const float *f, long out_h, long out_w,
                      long fh, long fw, double *out, double *abs_sum)
{
    if (bad_shape(out_h, out_w, fh, fw) || !in || !f || !out)
        return -1;
    const long pitch = out_w + fw - 1;
#pragma omp parallel for schedule(static)
    for (long y = 0; y < out_h; ++y) {
        for (long x = 0; x < out_w; ++x) {
            double v, a;
            one_point(in, f, pitch, fh, fw, y, x, &v, &a);
            out[y * out_w + x] = v;
            if (abs_sum)
                abs_sum[y * out_w + x] = a;
        }
    }
    return 0;
}

/* Selected output points (ys[k], xs[k]), k < n: the same definition, point by
 * point, for sampled checks at sizes where the full oracle is too slow.
 * Returns 0, or -1 on an invalid shape/pointer or a point out of range. */
int oracle_conv2d_points_f64(const float *in, const float *f, long out_h, long out_w,
                             long fh, long fw, const long *ys, const long *xs, long n,
                             double *out, double *abs_sum)
{
    if (bad_shape(out_h, out_w, fh, fw) || !in || !f || !ys || !xs || !out || n < 0)
        return -1;
    for (long k = 0; k < n; ++k)
        if (ys[k] < 0 || ys[k] >= out_h || xs[k] < 0 || xs[k] >= out_w)
            return -1;
    const long pitch = out_w + fw - 1;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
        double v, a;
        one_point(in, f, pitch, fh, fw, ys[k], xs[k], &v, &a);
        out[k] = v;
        if (abs_sum)
            abs_sum[k] = a;
    }
    return 0;
}

/* Rows [y0, y1) only (a horizontal band), written to out[(y-y0)*W + x]. */
int oracle_conv2d_rows_f64(const float *in, const float *f, long out_h, long out_w,
                           long fh, long fw, long y0, long y1, double *out, double *abs_sum)
{
    if (bad_shape(out_h, out_w, fh, fw) || !in || !f || !out || y0 < 0 || y1 > out_h || y0 > y1)
        return -1;
    const long pitch = out_w + fw - 1;
#pragma omp parallel for schedule(static)
    for (long y = y0; y < y1; ++y) {
        for (long x = 0; x < out_w; ++x) {
            double v, a;
            one_point(in, f, pitch, fh, fw, y, x, &v, &a);
            out[(y - y0) * out_w + x] = v;
            if (abs_sum)
                abs_sum[(y - y0) * out_w + x] = a;
        }
    }
    return 0;
}

/* Threads an OpenMP region of this library uses (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of later OpenMP regions (n >= 1; timing only: the
 * results do not depend on it, every output being one thread's sum). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
