// hos_fft.h -- FP64 complex FFT building blocks shared by the spectra
// kernels: small forward DFTs in registers, one self-sorting (Stockham)
// mixed-radix 8/4/2/3/5 stage over sequences held in LDS, and the radix
// plan (radix 8 first: fewer stages, so fewer LDS passes and barriers).
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
    int lg;      // log2(n) for a power of two, else -1 (index math by shifts)
    int r[16];
};

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Root i of the table (i < N <= 2^20): the byte offset is formed in 32 bits
// and added to the table's uniform base, one VALU op instead of a 64-bit
// address per load.
__device__ __attribute__((always_inline)) inline double2 tw_at(const double2 *__restrict__ tw,
                                                               int i)
{
    return *(const double2 *)((const char *)tw + (unsigned)i * 16u);
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
    } else if constexpr (R == 8) {
        // two 4-point DFTs (even, odd samples) joined by the eighth roots
        // of unity: X(p) = E(p) + w^p O(p), X(p+4) = E(p) - w^p O(p),
        // w = exp(-i pi/4) = c (1 - i)
        constexpr double c = 0.70710678118654752440;   // cos(pi/4)
        double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4>(e, tw, N);
        dft_small<4>(o, tw, N);
        const double2 t[4] = {o[0], make_double2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)),
                              make_double2(o[2].y, -o[2].x),
                              make_double2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y))};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = make_double2(e[q].x + t[q].x, e[q].y + t[q].y);
            v[q + 4] = make_double2(e[q].x - t[q].x, e[q].y - t[q].y);
        }
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
                double2 t = cmul(in[q], tw_at(tw, ((p * q) % R) * step));
                acc.x += t.x;
                acc.y += t.y;
            }
            v[p] = acc;
        }
    }
}

// LDS index of complex element i of an FFT area laid out with one padding
// element after every 2^PADSH (PADSH = 0: no padding).  The first radix-8
// stages write their outputs 8 or 64 elements apart; with a pad after every
// 8 elements (128 bytes) those strides no longer fall on the same LDS banks.
// An area of E elements then takes E + E / 2^PADSH slots.
template <int PADSH>
__device__ __attribute__((always_inline)) inline int lds_at(int i)
{
    return PADSH ? i + (i >> PADSH) : i;
}

template <int PADSH>
constexpr int lds_slots(int elems)
{
    return PADSH ? elems + (elems >> PADSH) : elems;
}

// THREADS: the workgroup size; ELEMS: the complex values of the caller's
// LDS area (CB * N <= ELEMS), which bounds the butterflies a thread holds.
// lgN, lgNs: log2 of N and Ns when N is a power of two (then so is Ns, and
// the butterfly indices come from shifts and masks), else -1.  PADSH: the
// area's padding (lds_at).
template <int R, int THREADS = FFT_THREADS, int ELEMS = FFT_LDS_ELEMS, int PADSH = 0>
__device__ inline void stockham_stage(double2 *sm, const double2 *__restrict__ tw, int N,
                                      int Ns, int CB, int lgN, int lgNs)
{
    constexpr int MAXIT = (ELEMS / R + THREADS - 1) / THREADS;
    constexpr int LGR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : -1;
    const int nbf = N / R, total = CB * nbf, stride = N / (Ns * R);
    const bool p2 = LGR > 0 && lgN >= 0;
    double2 v[MAXIT][R];
    int dst[MAXIT];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (u < total) {
            int cb, j, jq, k;
            if (p2) {
                cb = u >> (lgN - LGR);
                j = u & (nbf - 1);
                jq = j >> lgNs;
                k = j & (Ns - 1);
            } else {
                cb = u / nbf;
                j = u - cb * nbf;
                jq = j / Ns;
                k = j - jq * Ns;
            }
            dst[it] = cb * N + jq * Ns * R + k;
            const int src = cb * N + j;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                double2 x = sm[lds_at<PADSH>(src + q * nbf)];
                v[it][q] = q == 0 ? x : cmul(x, tw_at(tw, q * k * stride));
            }
            dft_small<R>(v[it], tw, N);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (u < total) {
#pragma unroll
            for (int p = 0; p < R; ++p)
                sm[lds_at<PADSH>(dst[it] + p * Ns)] = v[it][p];
        }
    }
    __syncthreads();
}

// One Stockham stage with every size known at compile time (N a power of
// two, CB sequences of it in LDS): the butterfly indices are shifts and
// masks of constants, and where NBF (resp. NS) is a multiple of the
// padding period the R padded LDS slots of a butterfly are one base plus
// constant offsets.  Same arithmetic as stockham_stage.
template <int R, int N, int NS, int CB, int THREADS, int PADSH>
__device__ inline void stockham_stage_c(double2 *sm, const double2 *__restrict__ tw)
{
    constexpr int NBF = N / R, TOTAL = CB * NBF, STRIDE = N / (NS * R);
    constexpr int MAXIT = (TOTAL + THREADS - 1) / THREADS;
    constexpr int P = 1 << PADSH;
    double2 v[MAXIT][R];
    int dst[MAXIT];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (TOTAL % THREADS == 0 || u < TOTAL) {
            const int cb = u / NBF, j = u % NBF, jq = j / NS, k = j % NS;
            dst[it] = cb * N + jq * NS * R + k;
            const int src = cb * N + j;
            const int base = lds_at<PADSH>(src);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int at = (PADSH && NBF % P == 0) ? base + q * NBF + ((q * NBF) >> PADSH)
                                                       : lds_at<PADSH>(src + q * NBF);
                const double2 x = sm[at];
                v[it][q] = q == 0 ? x : cmul(x, tw_at(tw, q * k * STRIDE));
            }
            dft_small<R>(v[it], tw, N);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int u = threadIdx.x + THREADS * it;
        if (TOTAL % THREADS == 0 || u < TOTAL) {
            const int base = lds_at<PADSH>(dst[it]);
#pragma unroll
            for (int p = 0; p < R; ++p) {
                const int at = (PADSH && NS % P == 0) ? base + p * NS + ((p * NS) >> PADSH)
                                                      : lds_at<PADSH>(dst[it] + p * NS);
                sm[at] = v[it][p];
            }
        }
    }
    __syncthreads();
}

// The stages of a compile-time power-of-two N from NS on, radix 8 first,
// then one 4 or 2 -- the radix order of factor(), so the results equal
// fft_lds's bit for bit.
template <int N, int NS, int CB, int THREADS, int PADSH>
__device__ inline void fft_lds_c(double2 *sm, const double2 *__restrict__ tw)
{
    if constexpr (NS < N) {
        constexpr int REM = N / NS;
        constexpr int R = REM % 8 == 0 ? 8 : REM % 4 == 0 ? 4 : 2;
        stockham_stage_c<R, N, NS, CB, THREADS, PADSH>(sm, tw);
        fft_lds_c<N, NS * R, CB, THREADS, PADSH>(sm, tw);
    }
}

inline FftRadices factor(int N)
{
    FftRadices f;
    f.n = N;
    f.lg = (N > 0 && (N & (N - 1)) == 0) ? __builtin_ctz((unsigned)N) : -1;
    int m = N, k = 0;
    while (m % 8 == 0) {
        f.r[k++] = 8;
        m /= 8;
    }
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

// POW2: N is a power of two (fr.lg >= 0), so only the radix 8/4/2 stages are
// compiled in -- the radix-3/5 butterflies need the most registers, and a
// kernel is allocated for its largest stage.
template <int THREADS = FFT_THREADS, int ELEMS = FFT_LDS_ELEMS, int PADSH = 0, bool POW2 = false>
__device__ inline void fft_lds(double2 *sm, const double2 *__restrict__ tw, const FftRadices &fr,
                               int CB)
{
    int Ns = 1, lgNs = 0;
    for (int st = 0; st < 16 && fr.r[st] > 0; ++st) {
        const int R = fr.r[st];
        if (R == 8)
            stockham_stage<8, THREADS, ELEMS, PADSH>(sm, tw, fr.n, Ns, CB, fr.lg, lgNs);
        else if (R == 4)
            stockham_stage<4, THREADS, ELEMS, PADSH>(sm, tw, fr.n, Ns, CB, fr.lg, lgNs);
        else if (R == 2 || POW2)
            stockham_stage<2, THREADS, ELEMS, PADSH>(sm, tw, fr.n, Ns, CB, fr.lg, lgNs);
        else if (R == 3)
            stockham_stage<3, THREADS, ELEMS, PADSH>(sm, tw, fr.n, Ns, CB, fr.lg, lgNs);
        else
            stockham_stage<5, THREADS, ELEMS, PADSH>(sm, tw, fr.n, Ns, CB, fr.lg, lgNs);
        Ns *= R;
        lgNs += R == 8 ? 3 : R == 4 ? 2 : R == 2 ? 1 : 0;
    }
}

}  // namespace hos
