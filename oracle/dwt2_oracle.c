/*
 * dwt2_oracle.c -- FP64 CPU oracle for the 2-D lifting DWT.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product library
 * (libdwt2.so) never calls it, and the two share no code, headers, tables or
 * constants: each side writes its own from the paper.
 *
 * Paper: D. Barina, M. Kula, P. Zemcik, "Parallel Wavelet Schemes for Images".
 *
 * What is computed.  The paper states that all of its 2-D lifting schemes give
 * exactly the result of ordinary separable lifting (Conclusions; the product
 * check S_U T_P = N_{P,U} in Sec. 3, "Monolithic Scheme").  So the oracle is
 * that plain definition, written out:
 *
 *   1-D: K predict/update pairs followed by the diagonal scaling step
 *        diag(zeta, 1/zeta)  (Sec. 2, "Lifting Scheme", the factorisation of M).
 *   2-D: Mallat's tensor-product decomposition (Sec. 2): the 1-D transform of
 *        every row, then of every column, giving the LL/HL/LH/HH quadrants.
 *   Multi-level: the next level transforms the LL quadrant (Sec. 1).
 *
 * Readings of points on which the paper is silent (each is listed in the
 * design notes of the repository):
 *   - Sample phase: L[n] = x[2n], H[n] = x[2n+1].  With this origin the
 *     paper's predict -1/2(1+z^-1) and update 1/4(1+z) (Sec. 5) read
 *     L[n], L[n+1] and H[n-1], H[n] respectively (an index relabelling of H);
 *     the DD 13/7 predict 1/16(z + z^-2) - 9/16(1 + z^-1) reads L[n-1..n+2]
 *     and its update 9/32(1 + z) - 1/32(z^-1 + z^2) reads H[n-2..n+1].
 *   - Borders: whole-sample symmetric extension, period 2(N-1), applied to
 *     the neighbour index of every lifting step.
 *   - Odd lengths: L gets ceil(N/2) samples, H gets floor(N/2); N >= 2.
 *   - Normalisation: PAPER scales L by zeta and H by 1/zeta in each 1-D pass
 *     (Sec. 2 and Sec. 5); the paper gives no zeta for DD 13/7, which is
 *     taken as sqrt(2), the value of the other interpolating transform (5/3),
 *     whose unscaled low-pass also has DC gain 1.  UNIT_DC instead scales L by 1/g and H by g, where g
 *     is the DC gain of the unscaled low-pass, so a constant image keeps its
 *     value in LL.  The two differ per 2-D subband by exact powers of two.
 *   - Inverse (not treated by the paper): per level, columns then rows; undo
 *     the scaling, then undo the pairs in reverse order, each update before
 *     its predict, with the same mirror.
 *
 * Output layout: Mallat layout of a W x H array (pitch W): LL in the top-left
 * ceil(H/2) x ceil(W/2) block, HL top-right, LH bottom-left, HH bottom-right,
 * recursive in LL.
 *
 * No blocking, fusion or reordering of the arithmetic: each lifting step
 * updates every sample of one parity from the nearest samples of the other
 * parity (two for CDF, four for DD 13/7), which is order-free, so the loops below may visit lines and
 * samples in any order (chosen only for cache-friendly memory access).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_SIZE (-2)
#define ORACLE_E_UNSUPPORTED (-3)
#define ORACLE_E_NOMEM (-7)

#define ORACLE_CDF53 0
#define ORACLE_CDF97 1
#define ORACLE_DD137 2

#define ORACLE_NORM_UNIT_DC 0
#define ORACLE_NORM_PAPER 1

/*
 * Each step is symmetric about the updated sample: in the interleaved signal
 * y (y[2n] = L[n], y[2n+1] = H[n]) a predict or update step at position i adds
 *   c1 (y[i-1] + y[i+1]) + c3 (y[i-3] + y[i+3]).
 */
typedef struct {
    int npairs;
    double predict[2], predict3[2]; /* c1, c3 of each predict step */
    double update[2], update3[2];   /* c1, c3 of each update step */
    double zeta;                    /* scaling factor of the paper's scaling step */
} lifting_t;

/*
 * Lifting factorisations (Sec. 5, "Evaluation").
 *
 * CDF 5/3: P(z) = -1/2 (1 + z^-1), U(z) = 1/4 (1 + z), zeta = sqrt(2).
 *
 * CDF 9/7: P0 = alpha(1+z^-1), U0 = beta(1+z), P1 = gamma(1+z^-1),
 * U1 = delta(1+z); the paper gives no values (it refers to Daubechies and
 * Sweldens).  The values below were derived at 40 digits: the 9-tap analysis
 * low-pass is sqrt(2) cos^4(w/2) q(sin^2(w/2)) and the 7-tap synthesis
 * low-pass is sqrt(2) cos^4(w/2) (1 - sin^2(w/2)/y_r), where
 * 1 + 4y + 10y^2 + 20y^3 = (1 - y/y_r) q(y) and y_r = -0.34238409485836913...
 * is its real root; alpha..delta and zeta follow from matching the lifting
 * impulse responses to those taps.  The tests re-derive them independently.
 */
static int get_lifting(int wavelet, lifting_t *w)
{
    memset(w, 0, sizeof(*w));
    if (wavelet == ORACLE_CDF53) {
        w->npairs = 1;
        w->predict[0] = -0.5;
        w->update[0] = 0.25;
        w->predict[1] = w->update[1] = 0.0;
        w->zeta = sqrt(2.0);
        return ORACLE_OK;
    }
    if (wavelet == ORACLE_CDF97) {
        w->npairs = 2;
        w->predict[0] = -1.58613434205992355842832;  /* alpha */
        w->update[0] = -0.0529801185729614146241296; /* beta  */
        w->predict[1] = 0.88291107553093329591979;   /* gamma */
        w->update[1] = 0.443506852043971152115604;   /* delta */
        w->zeta = 1.14960439886024115979508;
        return ORACLE_OK;
    }
    if (wavelet == ORACLE_DD137) {
        /* Sec. 5: P(z) = 1/16 (z + z^-2) - 9/16 (1 + z^-1),
         *         U(z) = 9/32 (1 + z) - 1/32 (z^-1 + z^2). */
        w->npairs = 1;
        w->predict[0] = -9.0 / 16.0;
        w->predict3[0] = 1.0 / 16.0;
        w->update[0] = 9.0 / 32.0;
        w->update3[0] = -1.0 / 32.0;
        w->zeta = sqrt(2.0);
        return ORACLE_OK;
    }
    return ORACLE_E_UNSUPPORTED;
}

/* DC gain of the unscaled low-pass: lift the constant signal 1. */
static double unscaled_dc_gain(const lifting_t *w)
{
    double L = 1.0, H = 1.0;
    for (int k = 0; k < w->npairs; k++) {
        H = H + w->predict[k] * (L + L) + w->predict3[k] * (L + L);
        L = L + w->update[k] * (H + H) + w->update3[k] * (H + H);
    }
    return L;
}

/* Per-1-D-pass scale factors of the L and H outputs. */
static int get_scales(int wavelet, int norm, double *s_lo, double *s_hi)
{
    lifting_t w;
    int st = get_lifting(wavelet, &w);
    if (st != ORACLE_OK) return st;
    if (norm == ORACLE_NORM_PAPER) {
        *s_lo = w.zeta;
        *s_hi = 1.0 / w.zeta;
    } else if (norm == ORACLE_NORM_UNIT_DC) {
        double g = unscaled_dc_gain(&w);
        *s_lo = 1.0 / g;
        *s_hi = g;
    } else {
        return ORACLE_E_UNSUPPORTED;
    }
    return ORACLE_OK;
}

/* Whole-sample symmetric mirror of index j into [0, n), period 2(n-1). */
static inline ptrdiff_t mirror(ptrdiff_t j, ptrdiff_t n)
{
    ptrdiff_t p = 2 * (n - 1);
    j %= p;
    if (j < 0) j += p;
    if (j >= n) j = p - j;
    return j;
}

/*
 * One lifting step on `lines` lines of length n stored in `a`:
 *   y[i] += c1 (y[m(i-1)] + y[m(i+1)]) + c3 (y[m(i-3)] + y[m(i+3)])
 * for every i with i % 2 == parity (the c3 term only when c3 != 0).
 * Samples of the updated parity read only samples of the other parity.
 * Rows (elem_stride == 1) loop lines outermost; columns (line_stride == 1)
 * loop sample positions outermost so that memory is walked row by row.
 */
static void lift_step(double *a, ptrdiff_t lines, ptrdiff_t n, ptrdiff_t line_stride,
                      ptrdiff_t elem_stride, int parity, double c1, double c3)
{
    if (elem_stride == 1) {
#pragma omp parallel for schedule(static)
        for (ptrdiff_t j = 0; j < lines; j++) {
            double *y = a + j * line_stride;
            for (ptrdiff_t i = parity; i < n; i += 2) {
                double d = c1 * (y[mirror(i - 1, n)] + y[mirror(i + 1, n)]);
                if (c3 != 0.0) d += c3 * (y[mirror(i - 3, n)] + y[mirror(i + 3, n)]);
                y[i] += d;
            }
        }
    } else {
#pragma omp parallel for schedule(static)
        for (ptrdiff_t i = parity; i < n; i += 2) {
            double *yi = a + i * elem_stride;
            const double *ym = a + mirror(i - 1, n) * elem_stride;
            const double *yp = a + mirror(i + 1, n) * elem_stride;
            const double *ym3 = a + mirror(i - 3, n) * elem_stride;
            const double *yp3 = a + mirror(i + 3, n) * elem_stride;
            for (ptrdiff_t j = 0; j < lines; j++) {
                double d = c1 * (ym[j * line_stride] + yp[j * line_stride]);
                if (c3 != 0.0) d += c3 * (ym3[j * line_stride] + yp3[j * line_stride]);
                yi[j * line_stride] += d;
            }
        }
    }
}

/*
 * Split each line into [L | H] (L = even samples, H = odd samples) and
 * scale them (forward), or the reverse (inverse).  tmp holds lines*n doubles.
 */
static void deinterleave(double *a, ptrdiff_t lines, ptrdiff_t n, ptrdiff_t line_stride,
                         ptrdiff_t elem_stride, double s_lo, double s_hi, double *tmp)
{
    ptrdiff_t nl = (n + 1) / 2;
#pragma omp parallel for schedule(static)
    for (ptrdiff_t j = 0; j < lines; j++) {
        double *t = tmp + j * n;
        const double *y = a + j * line_stride;
        for (ptrdiff_t i = 0; i < n; i++) {
            if (i % 2 == 0) t[i / 2] = y[i * elem_stride] * s_lo;
            else t[nl + i / 2] = y[i * elem_stride] * s_hi;
        }
    }
#pragma omp parallel for schedule(static)
    for (ptrdiff_t j = 0; j < lines; j++) {
        const double *t = tmp + j * n;
        double *y = a + j * line_stride;
        for (ptrdiff_t i = 0; i < n; i++) y[i * elem_stride] = t[i];
    }
}

static void interleave(double *a, ptrdiff_t lines, ptrdiff_t n, ptrdiff_t line_stride,
                       ptrdiff_t elem_stride, double s_lo, double s_hi, double *tmp)
{
    ptrdiff_t nl = (n + 1) / 2;
#pragma omp parallel for schedule(static)
    for (ptrdiff_t j = 0; j < lines; j++) {
        double *t = tmp + j * n;
        const double *y = a + j * line_stride;
        for (ptrdiff_t i = 0; i < n; i++) {
            if (i % 2 == 0) t[i] = y[(i / 2) * elem_stride] / s_lo;
            else t[i] = y[(nl + i / 2) * elem_stride] / s_hi;
        }
    }
#pragma omp parallel for schedule(static)
    for (ptrdiff_t j = 0; j < lines; j++) {
        const double *t = tmp + j * n;
        double *y = a + j * line_stride;
        for (ptrdiff_t i = 0; i < n; i++) y[i * elem_stride] = t[i];
    }
}

/* Forward 1-D transform of every line: lifting pairs, then split + scale. */
static void lines_forward(const lifting_t *w, double s_lo, double s_hi, double *a,
                          ptrdiff_t lines, ptrdiff_t n, ptrdiff_t line_stride,
                          ptrdiff_t elem_stride, double *tmp)
{
    for (int k = 0; k < w->npairs; k++) {
        lift_step(a, lines, n, line_stride, elem_stride, 1, w->predict[k], w->predict3[k]); /* H from L */
        lift_step(a, lines, n, line_stride, elem_stride, 0, w->update[k], w->update3[k]);   /* L from H */
    }
    deinterleave(a, lines, n, line_stride, elem_stride, s_lo, s_hi, tmp);
}

/* Inverse 1-D transform of every line: merge + unscale, then undo pairs. */
static void lines_inverse(const lifting_t *w, double s_lo, double s_hi, double *a,
                          ptrdiff_t lines, ptrdiff_t n, ptrdiff_t line_stride,
                          ptrdiff_t elem_stride, double *tmp)
{
    interleave(a, lines, n, line_stride, elem_stride, s_lo, s_hi, tmp);
    for (int k = w->npairs - 1; k >= 0; k--) {
        lift_step(a, lines, n, line_stride, elem_stride, 0, -w->update[k], -w->update3[k]);
        lift_step(a, lines, n, line_stride, elem_stride, 1, -w->predict[k], -w->predict3[k]);
    }
}

/* Level sizes: level k (0-based) transforms a wk x hk block; every wk, hk >= 2. */
static int level_sizes(int levels, int width, int height, int *ws, int *hs)
{
    if (levels < 1 || width < 1 || height < 1) return ORACLE_E_ARG;
    int w = width, h = height;
    for (int k = 0; k < levels; k++) {
        if (w < 2 || h < 2) return ORACLE_E_SIZE;
        ws[k] = w;
        hs[k] = h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    return ORACLE_OK;
}

#define ORACLE_MAX_LEVELS 32

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* The lifting constants the oracle uses: coef = {a_0, b_0, a_1, b_1}, the inner
 * taps c1 of each predict and update (DD 13/7 also has outer taps c3). */
int oracle_lifting_constants(int wavelet, int *npairs, double *coef, double *zeta)
{
    lifting_t w;
    int st = get_lifting(wavelet, &w);
    if (st != ORACLE_OK) return st;
    *npairs = w.npairs;
    for (int k = 0; k < w.npairs; k++) {
        coef[2 * k] = w.predict[k];
        coef[2 * k + 1] = w.update[k];
    }
    *zeta = w.zeta;
    return ORACLE_OK;
}

int oracle_scales(int wavelet, int norm, double *s_lo, double *s_hi)
{
    return get_scales(wavelet, norm, s_lo, s_hi);
}

/* 1-D forward transform of x[0..n) into y = [L | H]. */
int oracle_dwt1_forward(int wavelet, int norm, int n, const double *x, double *y)
{
    lifting_t w;
    double s_lo, s_hi;
    if (!x || !y) return ORACLE_E_ARG;
    if (n < 2) return ORACLE_E_SIZE;
    int st = get_lifting(wavelet, &w);
    if (st == ORACLE_OK) st = get_scales(wavelet, norm, &s_lo, &s_hi);
    if (st != ORACLE_OK) return st;
    double *tmp = malloc(sizeof(double) * (size_t)n);
    if (!tmp) return ORACLE_E_NOMEM;
    memcpy(y, x, sizeof(double) * (size_t)n);
    lines_forward(&w, s_lo, s_hi, y, 1, n, n, 1, tmp);
    free(tmp);
    return ORACLE_OK;
}

int oracle_dwt1_inverse(int wavelet, int norm, int n, const double *y, double *x)
{
    lifting_t w;
    double s_lo, s_hi;
    if (!x || !y) return ORACLE_E_ARG;
    if (n < 2) return ORACLE_E_SIZE;
    int st = get_lifting(wavelet, &w);
    if (st == ORACLE_OK) st = get_scales(wavelet, norm, &s_lo, &s_hi);
    if (st != ORACLE_OK) return st;
    double *tmp = malloc(sizeof(double) * (size_t)n);
    if (!tmp) return ORACLE_E_NOMEM;
    memcpy(x, y, sizeof(double) * (size_t)n);
    lines_inverse(&w, s_lo, s_hi, x, 1, n, n, 1, tmp);
    free(tmp);
    return ORACLE_OK;
}

/*
 * Multi-level 2-D forward DWT.  src and dst are width x height, row-major,
 * pitch = width; dst receives the Mallat layout.  dst may equal src.
 */
int oracle_dwt2_forward(int wavelet, int norm, int levels, int width, int height,
                        const double *src, double *dst)
{
    lifting_t w;
    double s_lo, s_hi;
    int ws[ORACLE_MAX_LEVELS], hs[ORACLE_MAX_LEVELS];
    if (!src || !dst) return ORACLE_E_ARG;
    if (levels > ORACLE_MAX_LEVELS) return ORACLE_E_SIZE;
    int st = level_sizes(levels, width, height, ws, hs);
    if (st == ORACLE_OK) st = get_lifting(wavelet, &w);
    if (st == ORACLE_OK) st = get_scales(wavelet, norm, &s_lo, &s_hi);
    if (st != ORACLE_OK) return st;
    size_t npx = (size_t)width * (size_t)height;
    double *tmp = malloc(sizeof(double) * npx);
    if (!tmp) return ORACLE_E_NOMEM;
    if (dst != src) memcpy(dst, src, sizeof(double) * npx);
    ptrdiff_t pitch = width;
    for (int k = 0; k < levels; k++) {
        /* rows: hs[k] lines of ws[k] samples */
        lines_forward(&w, s_lo, s_hi, dst, hs[k], ws[k], pitch, 1, tmp);
        /* columns: ws[k] lines of hs[k] samples */
        lines_forward(&w, s_lo, s_hi, dst, ws[k], hs[k], 1, pitch, tmp);
    }
    free(tmp);
    return ORACLE_OK;
}

/* Multi-level 2-D inverse DWT of a Mallat-layout array (pitch = width). */
int oracle_dwt2_inverse(int wavelet, int norm, int levels, int width, int height,
                        const double *src, double *dst)
{
    lifting_t w;
    double s_lo, s_hi;
    int ws[ORACLE_MAX_LEVELS], hs[ORACLE_MAX_LEVELS];
    if (!src || !dst) return ORACLE_E_ARG;
    if (levels > ORACLE_MAX_LEVELS) return ORACLE_E_SIZE;
    int st = level_sizes(levels, width, height, ws, hs);
    if (st == ORACLE_OK) st = get_lifting(wavelet, &w);
    if (st == ORACLE_OK) st = get_scales(wavelet, norm, &s_lo, &s_hi);
    if (st != ORACLE_OK) return st;
    size_t npx = (size_t)width * (size_t)height;
    double *tmp = malloc(sizeof(double) * npx);
    if (!tmp) return ORACLE_E_NOMEM;
    if (dst != src) memcpy(dst, src, sizeof(double) * npx);
    ptrdiff_t pitch = width;
    for (int k = levels - 1; k >= 0; k--) {
        lines_inverse(&w, s_lo, s_hi, dst, ws[k], hs[k], 1, pitch, tmp);
        lines_inverse(&w, s_lo, s_hi, dst, hs[k], ws[k], pitch, 1, tmp);
    }
    free(tmp);
    return ORACLE_OK;
}
