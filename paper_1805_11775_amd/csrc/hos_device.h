// hos_device.h -- small device helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hos {

// Parzen lag window d(m) with scale L (the lag-window reading of the
// smoothing step, Algorithm DBS's box smoothing): 1 - 6r^2 + 6r^3 for r = |m|/L <=
// 1/2, 2(1 - r)^3 for 1/2 < r <= 1, 0 beyond.  At L = 0 it is its L -> 0+
// limit: 1 at m = 0, 0 elsewhere.
__device__ inline double parzen_d(int m, int L)
{
    if (L == 0)
        return m == 0 ? 1.0 : 0.0;
    const double r = fabs((double)m) / (double)L;
    if (r <= 0.5)
        return 1.0 - 6.0 * r * r + 6.0 * r * r * r;
    if (r <= 1.0) {
        const double u = 1.0 - r;
        return 2.0 * u * u * u;
    }
    return 0.0;
}

// W3(w1, w2) = d(w1) d(w2) d(w1 - w2) (Parzen), d(w1) d(w2) (separable
// Parzen) or 1 (no window); `window` is an hos_window.
__device__ inline double window3(int w1, int w2, int M, int window)
{
    if (window == HOS_WIN_NONE)
        return 1.0;
    const double s = parzen_d(w1, M) * parzen_d(w2, M);
    return window == HOS_WIN_PARZEN ? s * parzen_d(w1 - w2, M) : s;
}

// c3(w1, w2) from the (M+1) x (M+1) table of third-order sums: the offsets
// {0, w1, w2} shifted by their minimum and sorted are {0, b, a}.  The lower
// triangle holds the fundamental region F of the hexagon, C[a][b] at
// [a][b] (b <= a <= M).  The square's corners (M < a <= 2M, a - M <= b <= M),
// present when amax = 2M, sit in the upper triangle: C[a][b] at [c][b] with
// c = a - M - 1 < b.  Lags with span a > amax give 0.
// The table entry of lag (w1, w2), not yet divided by n s^3.
__device__ inline double c3_table_sum(const double *__restrict__ cfull, int M, int amax, int w1,
                                      int w2)
{
    const int mn = min(0, min(w1, w2)), mx = max(0, max(w1, w2));
    const int a = mx - mn;
    if (a > amax)
        return 0.0;
    const int b = (w1 + w2) - mn - mx - mn;
    const int row = a <= M ? a : a - M - 1;
    return cfull[(int64_t)row * (M + 1) + b];
}

__device__ inline double c3_from_table(const double *__restrict__ cfull, int M, int amax,
                                       double norm, int w1, int w2)
{
    return c3_table_sum(cfull, M, amax, w1, w2) / norm;
}

// Fourth-order table helpers.  The lag pairs (a, b), 0 <= b <= a <= M, are
// numbered with b ascending, then a; pair_offset(M, b) is the first pair with
// second lag b.
__host__ __device__ inline int pair_offset(int M, int b)
{
    return b * (M + 1) - b * (b - 1) / 2;
}

__device__ inline void sort4(int *v)
{
#define SW(i, j)                 \
    if (v[i] > v[j]) {           \
        const int t_ = v[i];     \
        v[i] = v[j];             \
        v[j] = t_;               \
    }
    SW(0, 1) SW(2, 3) SW(0, 2) SW(1, 3) SW(1, 2)
#undef SW
}

// c4(t1,t2,t3), 0 outside {span <= M}.  Evaluated at the orbit's canonical
// member (c, b, a) -- the sorted offsets shifted to start at 0 -- so every
// member of an orbit gets the bitwise same value.
__device__ inline double c4_at(const double *__restrict__ m4tab, const double *__restrict__ c2,
                               int M, double norm4, int t1, int t2, int t3)
{
    int v[4] = {0, t1, t2, t3};
    sort4(v);
    const int a = v[3] - v[0];
    if (a > M)
        return 0.0;
    const int b = v[2] - v[0], c = v[1] - v[0];
    const int p = pair_offset(M, b) + (a - b);
    const double m4 = m4tab[(int64_t)p * (M + 1) + c] / norm4;
    return m4 - c2[c] * c2[a - b] - c2[b] * c2[a - c] - c2[a] * c2[b - c];
}

// Order five.  The fundamental region F5 = {0 <= d <= c <= b <= a <= M} is
// stored as rows (a, b, c) numbered with c ascending, and within one c as
// the pairs (a - c, b - c) of the lag range M - c; triple_offset(M, c) is
// the first row with smallest offset c.
__host__ __device__ inline int64_t triple_offset(int M, int c)
{
    // sum over k < c of (M - k + 1)(M - k + 2)/2 = S(M) - S(M - c), with
    // S(m) = (m + 1)(m + 2)(m + 3)/6 the number of pairs over lag ranges 0..m
    const int64_t a = M, b = (int64_t)M - c;
    return ((a + 1) * (a + 2) * (a + 3) - (b + 1) * (b + 2) * (b + 3)) / 6;
}

__device__ inline void sort5(int *v)
{
#define SW(i, j)                 \
    if (v[i] > v[j]) {           \
        const int t_ = v[i];     \
        v[i] = v[j];             \
        v[j] = t_;               \
    }
    SW(0, 1) SW(3, 4) SW(2, 4) SW(2, 3) SW(0, 3) SW(0, 2) SW(1, 4) SW(1, 3) SW(1, 2)
#undef SW
}

// c5(t1..t4), 0 outside {span <= M}: the fifth moment minus c2 * c3 over the
// ten ways to split the five offsets into a pair and a triple, evaluated at
// the orbit's canonical member (sorted offsets from 0) so that every member
// of an orbit gets the bitwise same value.  c3tab[a][b] (b <= a, stride
// M + 1) holds the final third-order cumulants.
__device__ inline double c5_at(const double *__restrict__ m5tab, const double *__restrict__ c2,
                               const double *__restrict__ c3tab, int M, double norm5, int t1,
                               int t2, int t3, int t4)
{
    int v[5] = {0, t1, t2, t3, t4};
    sort5(v);
    const int q[5] = {0, v[1] - v[0], v[2] - v[0], v[3] - v[0], v[4] - v[0]};
    const int a = q[4], b = q[3], c = q[2], d = q[1];
    if (a > M)
        return 0.0;
    const int64_t r = triple_offset(M, c) + pair_offset(M - c, b - c) + (a - b);
    double v5 = m5tab[r * (M + 1) + d] / norm5;
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int k = j + 1; k < 5; ++k) {
            int u[3], m = 0;
#pragma unroll
            for (int i = 0; i < 5; ++i)
                if (i != j && i != k)
                    u[m++] = q[i];
            v5 -= c2[q[k] - q[j]] * c3tab[(u[2] - u[0]) * (M + 1) + (u[1] - u[0])];
        }
    return v5;
}

// SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): a counter-based mix of z.
__device__ inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// v rounded to FP32 by stochastic rounding: up with probability equal to
// the fraction of the gap below v, down otherwise, the uniform draw being a
// deterministic function of `key` (the sample index).  Unlike round-to-
// nearest, the rounding error has zero mean for EVERY value, so rounding a
// centred series cannot leave a systematic offset (round-to-nearest of
// (x - mean) s has one: its error depends on the low bits of mean * s).
// Exact values, zero among them, are returned unchanged.
__device__ inline float round_stochastic_f32(double v, uint64_t key)
{
    const float f = (float)v;
    const double fd = (double)f;
    if (fd == v || !isfinite(v))
        return f;
    const float lo = fd < v ? f : nextafterf(f, -__builtin_huge_valf());
    const float hi = fd < v ? nextafterf(f, __builtin_huge_valf()) : f;
    const double frac = (v - (double)lo) / ((double)hi - (double)lo);
    const double u = (double)(splitmix64(key) >> 11) * 0x1.0p-53;
    return u < frac ? hi : lo;
}

}  // namespace hos
