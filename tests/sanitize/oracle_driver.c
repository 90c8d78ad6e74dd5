/* Exercise of the FP64 oracle's C core (test infrastructure) for the address
 * and undefined-behaviour sanitizers: every entry point on small records at
 * the edges of its index ranges -- the largest lag M = n - 1, lags whose
 * sums are empty, negative lags, one-sample records -- with output arrays
 * sized exactly as documented.  Checks two identities on the way (the c3
 * square is symmetric, the cube equals the point queries).  The prototypes
 * restate those of hos_oracle.c. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_center(const double *x, int64_t n, double *out);
void or_c3_at(const double *x, int64_t n, const int32_t *w1, const int32_t *w2, int64_t k,
              double *out);
void or_c3_square(const double *x, int64_t n, int32_t M, double *out);
void or_c2(const double *x, int64_t n, int32_t M, double *out);
void or_c4_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, int64_t k, double *out);
void or_c4_cube(const double *x, int64_t n, int32_t M, double *out);
void or_c5_at(const double *x, int64_t n, const int32_t *t1, const int32_t *t2,
              const int32_t *t3, const int32_t *t4, int64_t k, double *out);
void or_c5_hyper(const double *x, int64_t n, int32_t M, double *out);
void or_c3_grad(const double *x, int64_t n, int32_t M, const double *G, double *out);
void or_c3_grad_at(const double *x, int64_t n, int32_t M, const double *G, const int64_t *idx,
                   int64_t count, double *out);

static int failures = 0;

static void run(int64_t n, int32_t M)
{
    double *x = malloc(sizeof(double) * n), *xc = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i)
        x[i] = sin(1.7 * (double)i + 0.3) + 0.25 * (double)(i % 3);
    or_center(x, n, xc);
    const int64_t S = 2 * (int64_t)M + 1;
    double *sq = malloc(sizeof(double) * S * S);
    or_c3_square(xc, n, M, sq);
    for (int64_t a = 0; a < S; ++a)
        for (int64_t b = 0; b < S; ++b)
            if (fabs(sq[a * S + b] - sq[b * S + a]) > 1e-12)
                ++failures;
    double *c2 = malloc(sizeof(double) * (M + 1));
    or_c2(xc, n, M, c2);
    /* lags beyond the record: empty sums */
    int32_t w1[4] = {(int32_t)n, -(int32_t)n, M, -M}, w2[4] = {0, 1, -M, M};
    double o4[4];
    or_c3_at(xc, n, w1, w2, 4, o4);
    if (o4[0] != 0.0 || o4[1] != 0.0)
        ++failures;
    if (M <= 4) {
        const int64_t S3 = S * S * S;
        double *cube = malloc(sizeof(double) * S3);
        or_c4_cube(xc, n, M, cube);
        int32_t t1 = M, t2 = -M, t3 = 0;
        double v;
        or_c4_at(xc, n, &t1, &t2, &t3, 1, &v);
        if (fabs(v - cube[((int64_t)(2 * M) * S + 0) * S + M]) > 1e-12)
            ++failures;
        free(cube);
    }
    if (M <= 2) {
        double *hyper = malloc(sizeof(double) * S * S * S * S);
        or_c5_hyper(xc, n, M, hyper);
        int32_t t[4] = {M, -M, 0, M};
        double v;
        or_c5_at(xc, n, &t[0], &t[1], &t[2], &t[3], 1, &v);
        free(hyper);
    }
    double *G = malloc(sizeof(double) * S * S), *g = malloc(sizeof(double) * n);
    for (int64_t k = 0; k < S * S; ++k)
        G[k] = cos(0.1 * (double)k);
    or_c3_grad(xc, n, M, G, g);
    int64_t idx[3] = {0, n / 2, n - 1};
    double gs[3];
    or_c3_grad_at(xc, n, M, G, idx, 3, gs);
    for (int k = 0; k < 3; ++k)
        if (fabs(gs[k] - g[idx[k]]) > 1e-12 * (1.0 + fabs(g[idx[k]])))
            ++failures;
    free(x); free(xc); free(sq); free(c2); free(G); free(g);
}

int main(void)
{
    const int64_t ns[6] = {1, 2, 3, 7, 40, 257};
    for (int k = 0; k < 6; ++k) {
        const int64_t n = ns[k];
        const int32_t Ms[3] = {0, (int32_t)(n - 1 < 2 ? n - 1 : 2), (int32_t)(n - 1 < 9 ? n - 1 : 9)};
        for (int j = 0; j < 3; ++j)
            run(n, Ms[j]);
        run(n, (int32_t)(n - 1));
    }
    if (failures) {
        fprintf(stderr, "oracle driver: %d checks failed\n", failures);
        return 1;
    }
    printf("oracle driver: ok\n");
    return 0;
}
