/*
 * hos_oracle.c -- plain FP64 reference for the sample cumulants behind the
 * smoothed bispectrum / trispectrum estimators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the product path never
 * calls it.
 *
 * Every function below is the definition written out as a brute-force sum:
 * each lag is computed on its own, in natural index order, with no use of
 * the cumulant symmetries (so symmetry checks on its output are not
 * circular) and no blocking or reordering.  OpenMP only distributes
 * independent lags over threads; the arithmetic of one lag is sequential.
 *
 * Definitions (paper, Section 1 "Problem Statement": the k-th order moment
 * as the expectation of a product of k lagged samples; cumulants as
 * functions of the moments; ensemble averages replaced by time averages):
 *
 *   m3(w1,w2)    = (1/n) sum_t x_t x_{t+w1} x_{t+w2}
 *   m4(t1,t2,t3) = (1/n) sum_t x_t x_{t+t1} x_{t+t2} x_{t+t3}
 *   m5(t1..t4)   = (1/n) sum_t x_t x_{t+t1} x_{t+t2} x_{t+t3} x_{t+t4}
 *   c2(d)        = (1/n) sum_t x_t x_{t+d}
 *
 * where each sum runs over the t for which every index lies in [0, n)
 * (the same as zero padding outside the record) and x is the mean-removed
 * series, so c3 = m3.  The 1/n normalisation (a biased estimator) and the
 * index range are readings the paper leaves open.
 */
#include <stdint.h>
#include <stdlib.h>

static int64_t imax3(int64_t a, int64_t b, int64_t c)
{
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

static int64_t imin3(int64_t a, int64_t b, int64_t c)
{
    int64_t m = a < b ? a : b;
    return m < c ? m : c;
}

/* Plain FP64 mean removal: out_t = x_t - (sum_t x_t)/n, summed in order. */
void or_center(const double *x, int64_t n, double *out)
{
    double s = 0.0;
    for (int64_t t = 0; t < n; ++t)
        s += x[t];
    double mu = s / (double)n;
    for (int64_t t = 0; t < n; ++t)
        out[t] = x[t] - mu;
}

/* Third-order moment of x at one lag pair, sum over the valid t range. */
static double m3_one(const double *x, int64_t n, int64_t w1, int64_t w2)
{
    int64_t lo = -imin3(0, w1, w2);         /* all of t, t+w1, t+w2 >= 0 */
    int64_t hi = n - 1 - imax3(0, w1, w2);  /* all of them <= n-1        */
    double s = 0.0;
    for (int64_t t = lo; t <= hi; ++t)
        s += x[t] * x[t + w1] * x[t + w2];
    return s / (double)n;
}

/* c3 at `count` arbitrary lag pairs (w1[k], w2[k]). */
void or_c3_at(const double *x, int64_t n, const int32_t *w1, const int32_t *w2,
              int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = m3_one(x, n, w1[k], w2[k]);
}

/* c3 over the full square |w1|,|w2| <= M, row-major with lag w at w+M. */
void or_c3_square(const double *x, int64_t n, int32_t M, double *out)
{
    int64_t side = 2 * (int64_t)M + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < side; ++r)
        for (int64_t c = 0; c < side; ++c)
            out[r * side + c] = m3_one(x, n, r - M, c - M);
}

/* Second-order moment (= autocovariance of the centred series) at lag d. */
static double c2_one(const double *x, int64_t n, int64_t d)
{
    if (d < 0)
        d = -d;
    double s = 0.0;
    for (int64_t t = 0; t + d <= n - 1; ++t)
        s += x[t] * x[t + d];
    return s / (double)n;
}

/* c2(d) for d = 0..M. */
void or_c2(const double *x, int64_t n, int32_t M, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t d = 0; d <= M; ++d)
        out[d] = c2_one(x, n, d);
}

static double m4_one(const double *x, int64_t n, int64_t t1, int64_t t2, int64_t t3)
{
    int64_t mn = imin3(0, t1, t2 < t3 ? t2 : t3);  /* smallest of 0,t1,t2,t3 */
    int64_t mx = imax3(0, t1, t2 > t3 ? t2 : t3);  /* largest of 0,t1,t2,t3  */
    int64_t lo = -mn, hi = n - 1 - mx;
    double s = 0.0;
    for (int64_t t = lo; t <= hi; ++t)
        s += x[t] * x[t + t1] * x[t + t2] * x[t + t3];
    return s / (double)n;
}

/* Fourth-order moment at `count` lag triples. */
void or_m4_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = m4_one(x, n, t1[k], t2[k], t3[k]);
}

/*
 * Fourth-order cumulant of the zero-mean series at one lag triple: the
 * fourth moment minus the three pairings of second-order moments,
 *   c4 = m4(t1,t2,t3) - c2(t1) c2(t3-t2) - c2(t2) c2(t3-t1) - c2(t3) c2(t2-t1),
 * the moment-to-cumulant relation for four zero-mean variables
 * (X0,X1,X2,X3) = (x_t, x_{t+t1}, x_{t+t2}, x_{t+t3}).
 */
static double c4_one(const double *x, int64_t n, int64_t t1, int64_t t2, int64_t t3)
{
    double m4 = m4_one(x, n, t1, t2, t3);
    return m4 - c2_one(x, n, t1) * c2_one(x, n, t3 - t2)
              - c2_one(x, n, t2) * c2_one(x, n, t3 - t1)
              - c2_one(x, n, t3) * c2_one(x, n, t2 - t1);
}

void or_c4_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = c4_one(x, n, t1[k], t2[k], t3[k]);
}

/* c4 over the full cube |t1|,|t2|,|t3| <= M, index ((t1+M)*S + t2+M)*S + t3+M. */
void or_c4_cube(const double *x, int64_t n, int32_t M, double *out)
{
    int64_t S = 2 * (int64_t)M + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < S * S; ++r) {
        int64_t a = r / S, b = r % S;
        for (int64_t c = 0; c < S; ++c)
            out[r * S + c] = c4_one(x, n, a - M, b - M, c - M);
    }
}

/* Fifth-order moment at one lag quadruple. */
static double m5_one(const double *x, int64_t n, int64_t t1, int64_t t2, int64_t t3, int64_t t4)
{
    int64_t mn = 0, mx = 0;
    const int64_t t[4] = {t1, t2, t3, t4};
    for (int k = 0; k < 4; ++k) {
        if (t[k] < mn)
            mn = t[k];
        if (t[k] > mx)
            mx = t[k];
    }
    int64_t lo = -mn, hi = n - 1 - mx;
    double s = 0.0;
    for (int64_t i = lo; i <= hi; ++i)
        s += x[i] * x[i + t1] * x[i + t2] * x[i + t3] * x[i + t4];
    return s / (double)n;
}

void or_m5_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, const int32_t *t4, int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = m5_one(x, n, t1[k], t2[k], t3[k], t4[k]);
}

/*
 * Fifth-order cumulant of the zero-mean series at one lag quadruple: with
 * offsets o = (0, t1, t2, t3, t4) of the five variables X_k = x_{t+o_k},
 * the moment-to-cumulant relation for zero-mean variables keeps, besides
 * the fifth moment, only the partitions of {0..4} into a pair and a triple:
 *   c5 = m5 - sum over the ten pairs {j,k} of c2(o_k - o_j) m3(rest),
 * m3 of the remaining three offsets {p,q,r} taken relative to the first.
 */
static double c5_one(const double *x, int64_t n, int64_t t1, int64_t t2, int64_t t3, int64_t t4)
{
    const int64_t o[5] = {0, t1, t2, t3, t4};
    double c = m5_one(x, n, t1, t2, t3, t4);
    for (int j = 0; j < 5; ++j)
        for (int k = j + 1; k < 5; ++k) {
            int64_t r[3];
            int m = 0;
            for (int q = 0; q < 5; ++q)
                if (q != j && q != k)
                    r[m++] = o[q];
            c -= c2_one(x, n, o[k] - o[j]) * m3_one(x, n, r[1] - r[0], r[2] - r[0]);
        }
    return c;
}

void or_c5_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, const int32_t *t4, int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = c5_one(x, n, t1[k], t2[k], t3[k], t4[k]);
}

/* c5 over the hypercube |t_i| <= M, index (((t1+M)S + t2+M)S + t3+M)S + t4+M. */
void or_c5_hyper(const double *x, int64_t n, int32_t M, double *out)
{
    int64_t S = 2 * (int64_t)M + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < S * S; ++r) {
        int64_t a = r / S, b = r % S;
        for (int64_t c = 0; c < S; ++c)
            for (int64_t d = 0; d < S; ++d)
                out[(r * S + c) * S + d] = c5_one(x, n, a - M, b - M, c - M, d - M);
    }
}

/*
 * Gradient of a function of c3 with respect to the mean-removed series.
 * G is dF/dc3(w1,w2) over the square |w| <= M, row-major [(w1+M)(2M+1) +
 * (w2+M)].  Differentiating c3(w) = (1/n) sum_t x_t x_{t+w1} x_{t+w2} by x_j
 * gives one term for each of the three factors that can sit at j:
 *
 *   g_j = (1/n) sum_w G(w) [ x_{j+w1} x_{j+w2}          (t = j)
 *                          + x_{j-w1} x_{j-w1+w2}       (t + w1 = j)
 *                          + x_{j-w2} x_{j-w2+w1} ]     (t + w2 = j)
 *
 * with x = 0 outside [0, n) (the same index range as c3 itself).
 */
static double xz(const double *x, int64_t n, int64_t i)
{
    return (i >= 0 && i < n) ? x[i] : 0.0;
}

static double grad_one(const double *x, int64_t n, int32_t M, const double *G, int64_t j)
{
    const int64_t S = 2 * (int64_t)M + 1;
    double s = 0.0;
    for (int64_t w1 = -M; w1 <= M; ++w1)
        for (int64_t w2 = -M; w2 <= M; ++w2) {
            const double g = G[(w1 + M) * S + (w2 + M)];
            if (g == 0.0)
                continue;
            const double d = xz(x, n, j + w1) * xz(x, n, j + w2)
                           + xz(x, n, j - w1) * xz(x, n, j - w1 + w2)
                           + xz(x, n, j - w2) * xz(x, n, j - w2 + w1);
            s += g * d;
        }
    return s / (double)n;
}

void or_c3_grad(const double *x, int64_t n, int32_t M, const double *G, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < n; ++j)
        out[j] = grad_one(x, n, M, G, j);
}

/* The same at the sample indices idx[0..count). */
void or_c3_grad_at(const double *x, int64_t n, int32_t M, const double *G, const int64_t *idx,
                   int64_t count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k)
        out[k] = grad_one(x, n, M, G, idx[k]);
}
