// hos_fft.h -- FP64 complex FFT building blocks shared by the spectra
// kernels: small forward DFTs in registers, one self-sorting (Stockham)
// mixed-radix 4/2/3/5 stage over sequences held in LDS, and the radix plan.
//
// Transforms are unnormalised with the sign of Algorithm DBS's part DFT,
//     X(k) = sum_u x(u) exp(-2 pi i u k / N),
// and take their twiddles from a table of the N roots of unity.
#pragma once
#include <hip/hip_runtime.h>

namespace hos {

constexpr int FFT_THREADS = 256;
constexpr int FFT_LDS_ELEMS = 4096;   // complex doubles per workgroup (64 KB)

struct FftRadices {
    int n;
    int r[16];
};

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Forward DFT of size R in registers.
template <int R>
__device__ inline void dft_small(double2 *v, const double2 *__restrict__ tw, int N)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = make_double2(a.x + b.x, a.y + b.y);
        v[1] = make_double2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        double2 a = v[0], b = v[1], c = v[2], d = v[3];
        double2 s02 = make_double2(a.x + c.x, a.y + c.y), d02 = make_double2(a.x - c.x, a.y - c.y);
        double2 s13 = make_double2(b.x + d.x, b.y + d.y), d13 = make_double2(b.x - d.x, b.y - d.y);
        v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
        v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
        // -i * d13 = (d13.y, -d13.x)
        v[1] = make_double2(d02.x + d13.y, d02.y - d13.x);
        v[3] = make_double2(d02.x - d13.y, d02.y + d13.x);
    } else {
        double2 in[R];
#pragma unroll
        for (int q = 0; q < R; ++q)
            in[q] = v[q];
        const int step = N / R;
#pragma unroll
        for (int p = 0; p < R; ++p) {
            double2 acc = in[0];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                double2 t = cmul(in[q], tw[((p * q) % R) * step]);
                acc.x += t.x;
                acc.y += t.y;
            }
            v[p] = acc;
        }
    }
}

// THREADS: the workgroup size; ELEMS: the complex values of the caller's
// LDS area (CB * N <= ELEMS), which bounds the butterflies a thread holds.
template <int R, int THREADS = FFT_THREADS, int ELEMS = FFT_LDS_ELEMS>
__device__ inline void stockham_stage(double2 *sm, const double2 *__restrict__ tw, int N,
                                      int Ns, int CB)
{
    constexpr int MAXIT = (ELEMS / R + THREADS - 1) / THREADS;
    const int nbf = N / R, total = CB * nbf, stride = N / (Ns * R);
    double2 v[MAXIT][R];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (u < total) {
            const int cb = u / nbf, j = u - cb * nbf, k = j % Ns;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                double2 x = sm[cb * N + j + q * nbf];
                v[it][q] = q == 0 ? x : cmul(x, tw[q * k * stride]);
            }
            dft_small<R>(v[it], tw, N);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (u < total) {
            const int cb = u / nbf, j = u - cb * nbf, k = j % Ns;
            const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int p = 0; p < R; ++p)
                sm[cb * N + idxD + p * Ns] = v[it][p];
        }
    }
    __syncthreads();
}

inline FftRadices factor(int N)
{
    FftRadices f;
    f.n = N;
    int m = N, k = 0;
    while (m % 4 == 0) {
        f.r[k++] = 4;
        m /= 4;
    }
    while (m % 2 == 0) {
        f.r[k++] = 2;
        m /= 2;
    }
    while (m % 3 == 0) {
        f.r[k++] = 3;
        m /= 3;
    }
    while (m % 5 == 0) {
        f.r[k++] = 5;
        m /= 5;
    }
    for (; k < 16; ++k)
        f.r[k] = 0;
    return f;
}

template <int THREADS = FFT_THREADS, int ELEMS = FFT_LDS_ELEMS>
__device__ inline void fft_lds(double2 *sm, const double2 *__restrict__ tw, const FftRadices &fr,
                               int CB)
{
    int Ns = 1;
    for (int st = 0; st < 16 && fr.r[st] > 0; ++st) {
        const int R = fr.r[st];
        if (R == 4)
            stockham_stage<4, THREADS, ELEMS>(sm, tw, fr.n, Ns, CB);
        else if (R == 2)
            stockham_stage<2, THREADS, ELEMS>(sm, tw, fr.n, Ns, CB);
        else if (R == 3)
            stockham_stage<3, THREADS, ELEMS>(sm, tw, fr.n, Ns, CB);
        else
            stockham_stage<5, THREADS, ELEMS>(sm, tw, fr.n, Ns, CB);
        Ns *= R;
    }
}

}  // namespace hos
