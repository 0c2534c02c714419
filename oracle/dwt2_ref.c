/*
 * Reference 2-D discrete wavelet transform, FP64, plain separable lifting.
 *
 * TEST INFRASTRUCTURE. This file is the oracle that the GPU library is checked
 * against. Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it. It shares no code, header or constant with the GPU
 * library and the GPU library never calls it.
 *
 * What it computes (Barina et al., "Accelerating Discrete Wavelet Transforms
 * on GPUs"):
 *   - the 1-D transform as a sequence of lifting pairs, a predict P followed by
 *     an update U (Sec. 2, eq. 2), for CDF 5/3 and CDF 9/7 (Sec. 3, Table 1);
 *   - the 2-D transform as the tensor product of 1-D transforms, applied along
 *     rows (horizontal axis m) and then along columns (vertical axis n)
 *     (Sec. 2, the separable schemes; H and V steps may be interleaved in any
 *     order because the filters are linear, so rows-then-columns gives the same
 *     result as the paper's per-pair interleaving);
 *   - the multi-level transform by recursion on the low-low band (dyadic
 *     pyramid, Mallat layout). The paper leaves multi-scale to future work
 *     (Sec. 5); the recursion is the standard reading.
 *   - the inverse, by running the same steps in reverse order with negated
 *     coefficients and reciprocal scaling.
 *
 * Readings where the paper is silent (each one is checked by the pins in
 * tests/test_oracle_*.py, never by this file itself):
 *   - Lifting constants: the standard factorisation of the CDF 9/7 pair
 *     (alpha, beta, gamma, delta, K) and the 5/3 pair (-1/2, 1/4). The paper
 *     cites them without printing them.
 *   - Phase: pixel 0 is an even sample. A predict adds p times the even
 *     neighbours at 2i and 2i+2 to the odd sample 2i+1 (P = p(1+z)); an update
 *     adds u times the odd neighbours at 2i-1 and 2i+1 to the even sample 2i
 *     (U = u(1+z^-1)).
 *   - Boundary: whole-sample symmetric extension, x[-k] = x[k] and
 *     x[N-1+k] = x[N-1-k]. Inside the lifting steps this is s[N/2] = s[N/2-1]
 *     at the right end and d[-1] = d[0] at the left end.
 *   - Scaling: unit gain. The low band is divided by K and the high band is
 *     multiplied by K/2 (9/7); the 5/3 high band is halved. The analysis
 *     low-pass then has DC gain 1 and the high-pass has Nyquist gain 1.
 *   - Layout: one W x H buffer. After level j the low-low band of size
 *     (W/2^j) x (H/2^j) sits at the top-left, HL (horizontal high) to its right,
 *     LH below it and HH diagonally.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_INVALID_ARG (-1)

enum { ORACLE_CDF97 = 0, ORACLE_CDF53 = 1 };

typedef struct {
    int npairs;
    double p[2];   /* predict coefficient of each pair, in the order applied */
    double u[2];   /* update coefficient of each pair */
    double zl;     /* scaling of the low (even) phase */
    double zh;     /* scaling of the high (odd) phase */
} oracle_wavelet;

static int oracle_get_wavelet(int w, oracle_wavelet *out)
{
    if (w == ORACLE_CDF97) {
        const double K = 1.230174104914001;
        out->npairs = 2;
        out->p[0] = -1.586134342059924;   /* alpha */
        out->u[0] = -0.052980118572961;   /* beta  */
        out->p[1] = 0.882911075530934;    /* gamma */
        out->u[1] = 0.443506852043971;    /* delta */
        out->zl = 1.0 / K;
        out->zh = K / 2.0;
        return 0;
    }
    if (w == ORACLE_CDF53) {
        out->npairs = 1;
        out->p[0] = -0.5;
        out->u[0] = 0.25;
        out->p[1] = 0.0;
        out->u[1] = 0.0;
        out->zl = 1.0;
        out->zh = 0.5;
        return 0;
    }
    return -1;
}

/* Forward 1-D transform of n (even) samples x[0], x[stride], ... in place:
 * on return the first n/2 positions hold the low band and the last n/2 the
 * high band. tmp holds n doubles. */
static void fwd_line(double *x, int n, int64_t stride, double *tmp,
                     const oracle_wavelet *wv)
{
    const int h = n / 2;
    double *s = tmp, *d = tmp + h;
    for (int i = 0; i < h; ++i) {
        s[i] = x[(int64_t)(2 * i) * stride];
        d[i] = x[(int64_t)(2 * i + 1) * stride];
    }
    for (int k = 0; k < wv->npairs; ++k) {
        const double p = wv->p[k], u = wv->u[k];
        for (int i = 0; i < h; ++i) {
            const double right = (i + 1 < h) ? s[i + 1] : s[h - 1];
            d[i] += p * (s[i] + right);
        }
        for (int i = 0; i < h; ++i) {
            const double left = (i > 0) ? d[i - 1] : d[0];
            s[i] += u * (left + d[i]);
        }
    }
    for (int i = 0; i < h; ++i) {
        x[(int64_t)i * stride] = s[i] * wv->zl;
        x[(int64_t)(h + i) * stride] = d[i] * wv->zh;
    }
}

/* Inverse of fwd_line. */
static void inv_line(double *x, int n, int64_t stride, double *tmp,
                     const oracle_wavelet *wv)
{
    const int h = n / 2;
    double *s = tmp, *d = tmp + h;
    for (int i = 0; i < h; ++i) {
        s[i] = x[(int64_t)i * stride] / wv->zl;
        d[i] = x[(int64_t)(h + i) * stride] / wv->zh;
    }
    for (int k = wv->npairs - 1; k >= 0; --k) {
        const double p = wv->p[k], u = wv->u[k];
        for (int i = 0; i < h; ++i) {
            const double left = (i > 0) ? d[i - 1] : d[0];
            s[i] -= u * (left + d[i]);
        }
        for (int i = 0; i < h; ++i) {
            const double right = (i + 1 < h) ? s[i + 1] : s[h - 1];
            d[i] -= p * (s[i] + right);
        }
    }
    for (int i = 0; i < h; ++i) {
        x[(int64_t)(2 * i) * stride] = s[i];
        x[(int64_t)(2 * i + 1) * stride] = d[i];
    }
}

/* One level on the top-left w x h region of a buffer with row pitch `pitch`. */
static int level_2d(double *buf, int w, int h, int64_t pitch,
                    const oracle_wavelet *wv, int inverse, int nthreads)
{
    const int nmax = (w > h) ? w : h;
    int failed = 0;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *tmp = (double *)malloc(sizeof(double) * (size_t)nmax);
        if (!tmp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        }
        if (!inverse) {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int r = 0; r < h; ++r)
                if (tmp) fwd_line(buf + (int64_t)r * pitch, w, 1, tmp, wv);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int c = 0; c < w; ++c)
                if (tmp) fwd_line(buf + c, h, pitch, tmp, wv);
        } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int c = 0; c < w; ++c)
                if (tmp) inv_line(buf + c, h, pitch, tmp, wv);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int r = 0; r < h; ++r)
                if (tmp) inv_line(buf + (int64_t)r * pitch, w, 1, tmp, wv);
        }
        free(tmp);
    }
    return failed ? ORACLE_ERR_INVALID_ARG : ORACLE_OK;
}

static int check_args(const void *a, const void *b, int W, int H, int wavelet,
                      int levels, oracle_wavelet *wv)
{
    if (!a || !b || W < 2 || H < 2 || levels < 1 || levels > 30)
        return ORACLE_ERR_INVALID_ARG;
    if (oracle_get_wavelet(wavelet, wv) != 0) return ORACLE_ERR_INVALID_ARG;
    if ((W % (1 << levels)) != 0 || (H % (1 << levels)) != 0)
        return ORACLE_ERR_INVALID_ARG;
    return ORACLE_OK;
}

/* Forward L-level 2-D DWT: src (W x H, contiguous) -> coef (Mallat layout). */
int oracle_dwt2_forward(const double *src, double *coef, int W, int H,
                        int wavelet, int levels, int nthreads)
{
    oracle_wavelet wv;
    int st = check_args(src, coef, W, H, wavelet, levels, &wv);
    if (st) return st;
    if (nthreads < 1) nthreads = 1;
    if (coef != src) memmove(coef, src, sizeof(double) * (size_t)W * (size_t)H);
    for (int j = 0; j < levels; ++j) {
        st = level_2d(coef, W >> j, H >> j, W, &wv, 0, nthreads);
        if (st) return st;
    }
    return ORACLE_OK;
}

/* Inverse L-level 2-D DWT: coef (Mallat layout) -> dst (W x H). */
int oracle_dwt2_inverse(const double *coef, double *dst, int W, int H,
                        int wavelet, int levels, int nthreads)
{
    oracle_wavelet wv;
    int st = check_args(coef, dst, W, H, wavelet, levels, &wv);
    if (st) return st;
    if (nthreads < 1) nthreads = 1;
    if (dst != coef) memmove(dst, coef, sizeof(double) * (size_t)W * (size_t)H);
    for (int j = levels - 1; j >= 0; --j) {
        st = level_2d(dst, W >> j, H >> j, W, &wv, 1, nthreads);
        if (st) return st;
    }
    return ORACLE_OK;
}

/* 1-D transforms of one even-length signal, for impulse-response pins.
 * Output: low band in x[0..n/2), high band in x[n/2..n). */
int oracle_dwt1_forward(double *x, int n, int wavelet)
{
    oracle_wavelet wv;
    if (!x || n < 2 || (n & 1) || oracle_get_wavelet(wavelet, &wv) != 0)
        return ORACLE_ERR_INVALID_ARG;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!tmp) return ORACLE_ERR_INVALID_ARG;
    fwd_line(x, n, 1, tmp, &wv);
    free(tmp);
    return ORACLE_OK;
}

int oracle_dwt1_inverse(double *x, int n, int wavelet)
{
    oracle_wavelet wv;
    if (!x || n < 2 || (n & 1) || oracle_get_wavelet(wavelet, &wv) != 0)
        return ORACLE_ERR_INVALID_ARG;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!tmp) return ORACLE_ERR_INVALID_ARG;
    inv_line(x, n, 1, tmp, &wv);
    free(tmp);
    return ORACLE_OK;
}

/* Number of OpenMP threads the oracle would use for a request of n (0 = all). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
