// k_c4.hip -- fourth-order cumulant (trispectrum path) on the matrix cores.
//
// The paper extends its bispectrum algorithms to the trispectrum (Section 1;
// Section 3 states the k-th order generalisation).  The fourth-order sample
// moment of the mean-removed series over its fundamental region
// F4 = {0 <= c <= b <= a <= M},
//     C4[a][b][c] = sum_i x_i x_{i+a} x_{i+b} x_{i+c},
// is a contraction over the sample index i whose rows are the lag pairs
// (a, b): the product row Y_ab[i] = x_i x_{i+a} x_{i+b} meets the Hankel
// operand T[i][c] = x_{i+c}, for c <= b.  Pairs are numbered with b
// ascending (then a), so a block of 32 consecutive pairs spans few values of
// b and needs only ceil((b_max + 1) / 32) column blocks.
//
// The cumulant follows from the moments by the zero-mean moment-to-cumulant
// relation (Section 1: cumulants are functions of the moments),
//     c4(t1,t2,t3) = m4 - c2(t1) c2(t3-t2) - c2(t2) c2(t3-t1) - c2(t3) c2(t2-t1),
// with the second-order moments c2(d) = (1/n) sum_i x_i x_{i+d} taken in FP64
// from the input.  Every lag triple maps onto F4 by shifting the four sample
// offsets {0, t1, t2, t3} by their minimum and sorting (the 24-fold symmetry).
//
// Arithmetic, staging and precision handling follow the c3 contraction:
// FP32 (32x32x2) or FP16/BF16 hi+lo (32x32x16, three products) on the matrix
// cores, FP32 accumulation flushed to FP64, FP64 partials summed in a fixed
// order.  One workgroup = 4 waves = 4 pair blocks over a contiguous range of
// 512-sample chunks; all pair blocks read the same staged window of x.
#include <algorithm>

#include "hos_internal.h"
#include "hos_device.h"
#include "hos_fft.h"

namespace hos {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline void unpack8(float4 a, float4 b, float *v)
{
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// (a, b) of pair p; M + 1 - b pairs share each b.
__device__ inline void pair_ab(int M, int p, int &a, int &b)
{
    int bb = 0;
    while (bb < M && pair_offset(M, bb + 1) <= p)
        ++bb;
    b = bb;
    a = bb + (p - pair_offset(M, bb));
}

// (a, b, c) of order-five row r: rows with smallest offset c come in the
// pair order of the lag range M - c, shifted by c.
__device__ inline void triple_abc(int M, int r, int &a, int &b, int &c)
{
    int cc = 0;
    while (cc < M && triple_offset(M, cc + 1) <= r)
        ++cc;
    int ap, bp;
    pair_ab(M - cc, r - (int)triple_offset(M, cc), ap, bp);
    a = ap + cc;
    b = bp + cc;
    c = cc;
}

// Row r of the order-ORD contraction: the lag offsets whose samples multiply
// x_i (a, b for order four; a, b, c for order five) and the bound of its
// Hankel columns (the smallest offset: b, resp. c).
template <int ORD>
__device__ inline void row_offsets(int M, int r, int &a, int &b, int &c, int &bound)
{
    if constexpr (ORD == 4) {
        pair_ab(M, r, a, b);
        c = 0;
        bound = b;
    } else {
        triple_abc(M, r, a, b, c);
        bound = c;
    }
}

template <int PATH>
struct C4Ops;

template <>
struct C4Ops<HOS_PATH_SPLIT_FP16> {
    typedef halfx8 vec;
    // hi = RNE16(fl32(p q)), lo = RNE16(p q - hi) from the exact product
    // (see the c3 split)
    __device__ static inline void split(const float *p, const float *q, vec &h, vec &l)
    {
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t hv, lv;
            const float y0 = p[2 * k] * q[2 * k], y1 = p[2 * k + 1] * q[2 * k + 1];
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hv) : "v"(y0), "v"(y1));
            asm("v_fma_mixlo_f16 %0, %1, %2, -%3 op_sel_hi:[0,0,1]"
                : "=v"(lv) : "v"(p[2 * k]), "v"(q[2 * k]), "v"(hv));
            asm("v_fma_mixhi_f16 %0, %1, %2, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
                : "+v"(lv) : "v"(p[2 * k + 1]), "v"(q[2 * k + 1]), "v"(hv));
            hw[k] = hv;
            lw[k] = lv;
        }
        h = __builtin_bit_cast(vec, hw);
        l = __builtin_bit_cast(vec, lw);
    }
    __device__ static inline floatx16 mma(vec a, vec b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct C4Ops<HOS_PATH_SPLIT_BF16> {
    typedef bf16x8 vec;
    __device__ static inline void split(const float *p, const float *q, vec &h, vec &l)
    {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            __bf16 hh = (__bf16)(p[j] * q[j]);
            h[j] = hh;
            l[j] = (__bf16)__builtin_fmaf(p[j], q[j], -(float)hh);
        }
    }
    __device__ static inline floatx16 mma(vec a, vec b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// Keeps an FP64 running sum in accumulation registers (split paths: the
// operand and staging registers fill the vector file).
__device__ __attribute__((always_inline)) inline void pin_agpr(double &v)
{
    asm volatile("" : "+a"(v));
}

constexpr int C4_MAX_NCB = (C4_MAX_M + 1 + 31) / 32;   // column blocks per pair block

template <int PATH, int WX>
struct C4Lds {
    static constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    static constexpr int WLEN = KC + WX;
    static constexpr int NXI = KC / 4;
    // split paths: the FP16/BF16 hi and lo tables of the window; the FP32
    // path reads its Hankel operand from xw
    static constexpr int NXB = SPLIT ? 2 * WLEN : 0;
    static constexpr int TOTAL = NXI + WLEN + NXB;
    static constexpr int NCH = TOTAL / 64;
    static constexpr int NPW = (NCH + 3) / 4;
    static_assert(WLEN % 64 == 0, "window must be wave-chunk aligned");
    float4 xi[NXI];
    float4 xw[WLEN];            // x window table: entry o = x[i0 + o .. i0 + o + 3]
    uint4 xb[SPLIT ? NXB : 1];  // hi, then lo window tables of the same range
};

template <int PATH, int WX, int NPW = C4Lds<PATH, WX>::NPW>
__device__ __attribute__((always_inline)) inline void
c4_load(u32x4 (&stg)[NPW], const float *__restrict__ xf,
        const uint4 *__restrict__ win4, const uint4 *__restrict__ win8h,
        const uint4 *__restrict__ win8l, int64_t i0, int wave, int lane)
{
    typedef C4Lds<PATH, WX> CL;
    const u32x4 *xf4 = (const u32x4 *)xf, *w4 = (const u32x4 *)win4,
                *w8h = (const u32x4 *)win8h, *w8l = (const u32x4 *)win8l;
#pragma unroll
    for (int m = 0; m < CL::NPW; ++m) {
        const int j = wave + 4 * m, e = 64 * j;
        const u32x4 *src;
        if (e < CL::NXI)
            src = xf4 + (i0 >> 2) + e;
        else if (e < CL::NXI + CL::WLEN)
            src = w4 + i0 + (e - CL::NXI);
        else {
            const int e2 = e - CL::NXI - CL::WLEN;
            if (e2 < CL::WLEN)
                src = w8h + i0 + e2;
            else
                src = w8l + i0 + (e2 - CL::WLEN);
        }
        if (j < CL::NCH)
            stg[m] = src[lane];
    }
}

// neg: store the x_i run with its sign flipped.  Odd chunks run on -x_i and
// are flushed with a minus sign, which cancels the matrix cores' directed
// (toward -infinity) rounding bias between chunks.
template <int PATH, int WX, int NPW = C4Lds<PATH, WX>::NPW>
__device__ __attribute__((always_inline)) inline void
c4_store(const u32x4 (&stg)[NPW], C4Lds<PATH, WX> &L, int wave, int lane, bool neg)
{
    typedef C4Lds<PATH, WX> CL;
    u32x4 *base = (u32x4 *)&L;
    const unsigned flip = neg ? 0x80000000u : 0u;
#pragma unroll
    for (int m = 0; m < CL::NPW; ++m) {
        const int j = wave + 4 * m;
        if (j < CL::NCH)
            base[64 * j + lane] = 64 * j < CL::NXI ? (stg[m] ^ flip) : stg[m];
    }
}

// One chunk for one wave: row block rows (lane rl holds row (a, b[, c]))
// against NCOL column blocks.  Order
// four: product row x_i x_{i+a} x_{i+b}; order five: x_i x_{i+a} x_{i+b}
// x_{i+c}; its last factor is split from the exact FP32 product.
template <int ORD, int PATH, int WX, int NCOL>
__device__ __attribute__((always_inline)) inline void c4_chunk(const C4Lds<PATH, WX> &L, int a, int b, int c,
                                int rl, int h, floatx16 (&acc)[NCOL],
                                double (&acc64)[NCOL][16], float sgn)
{
    constexpr int NG = KC / GROUP;
    constexpr int WLEN = C4Lds<PATH, WX>::WLEN;
#pragma unroll 2
    for (int g = 0; g < NG; ++g) {
        const int ib = g * GROUP + 8 * h;
        float xi[8], xa[8], xb[8], p[8];
        unpack8(L.xi[ib >> 2], L.xi[(ib >> 2) + 1], xi);
        unpack8(L.xw[ib + a], L.xw[ib + a + 4], xa);
        unpack8(L.xw[ib + b], L.xw[ib + b + 4], xb);
        // rows past the last pair compute with a = b = 0 and are never
        // read back (the reduction keeps rows r < P only)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            p[j] = xi[j] * xa[j];
        if constexpr (ORD == 5) {
            // x_{i+b} joins the product; x_{i+c} is the last factor
            float xc[8];
            unpack8(L.xw[ib + c], L.xw[ib + c + 4], xc);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                p[j] *= xb[j];
                xb[j] = xc[j];
            }
        }
        if constexpr (PATH == HOS_PATH_FP32) {
            float y[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                y[j] = p[j] * xb[j];
#pragma unroll
            for (int cb = 0; cb < NCOL; ++cb) {
                const int o = ib + 32 * cb + rl;
                float t[8];
                unpack8(L.xw[o], L.xw[o + 4], t);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(y[j], t[j], acc[cb], 0, 0, 0);
            }
            if ((g & 3) == 3) {
#pragma unroll
                for (int cb = 0; cb < NCOL; ++cb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        acc64[cb][v] += (double)(sgn * acc[cb][v]);
                        acc[cb][v] = 0.0f;
                    }
            }
        } else {
            typedef C4Ops<PATH> Ops;
            typename Ops::vec yh, yl;
            Ops::split(p, xb, yh, yl);
#pragma unroll
            for (int cb = 0; cb < NCOL; ++cb) {
                const int o = ib + 32 * cb + rl;
                const typename Ops::vec th = __builtin_bit_cast(typename Ops::vec, L.xb[o]);
                const typename Ops::vec tl = __builtin_bit_cast(typename Ops::vec, L.xb[WLEN + o]);
                acc[cb] = Ops::mma(yh, th, acc[cb]);
                acc[cb] = Ops::mma(yh, tl, acc[cb]);
                acc[cb] = Ops::mma(yl, th, acc[cb]);
            }
        }
    }
    if constexpr (PATH != HOS_PATH_FP32) {
#pragma unroll
        for (int cb = 0; cb < NCOL; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc64[cb][v] += (double)(sgn * acc[cb][v]);
                pin_agpr(acc64[cb][v]);
                acc[cb][v] = 0.0f;
            }
    }
}

// The chunk loop of one workgroup with NCOL column blocks per wave (uniform
// over the workgroup, so every wave takes the same instantiation and meets
// the same barriers).
template <int ORD, int PATH, int WX, int NCOL>
__device__ __attribute__((always_inline)) inline void c4_run(C4Lds<PATH, WX> (&buf)[2], const float *__restrict__ xf,
                              const uint4 *__restrict__ win4, const uint4 *__restrict__ win8h,
                              const uint4 *__restrict__ win8l, double *__restrict__ part,
                              int a, int b, int c3, int rb, int s, int RB, int NCB,
                              int64_t c0, int64_t c1, int wave, int lane)
{
    const int rl = lane & 31, h = lane >> 5;
    floatx16 acc[NCOL];
    double acc64[NCOL][16];
#pragma unroll
    for (int cb = 0; cb < NCOL; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc[cb][v] = 0.0f;
            acc64[cb][v] = 0.0;
            if constexpr (PATH != HOS_PATH_FP32)
                pin_agpr(acc64[cb][v]);
        }

    u32x4 stg[C4Lds<PATH, WX>::NPW];
    c4_load<PATH, WX>(stg, xf, win4, win8h, win8l, c0 * KC, wave, lane);
    c4_store<PATH, WX>(stg, buf[0], wave, lane, c0 & 1);
    __syncthreads();
    int cur = 0;
    for (int64_t c = c0; c < c1; ++c) {
        const bool has_next = c + 1 < c1;
        if (has_next)
            c4_load<PATH, WX>(stg, xf, win4, win8h, win8l, (c + 1) * KC, wave, lane);
        c4_chunk<ORD, PATH, WX, NCOL>(buf[cur], a, b, c3, rl, h, acc, acc64,
                                      (c & 1) ? -1.0f : 1.0f);
        if (!has_next)
            break;
        cur ^= 1;
        c4_store<PATH, WX>(stg, buf[cur], wave, lane, (c + 1) & 1);
        __syncthreads();
    }
    if (rb < RB) {
#pragma unroll
        for (int cb = 0; cb < NCOL; ++cb) {
            double *dst = part + (((int64_t)s * RB + rb) * NCB + cb) * 1024;
#pragma unroll
            for (int v = 0; v < 16; ++v)
                dst[v * 64 + lane] = acc64[cb][v];
        }
    }
}

// Grid (ceil(RB/4), S): workgroup (x, s) runs row blocks 4x .. 4x+3 over
// chunks [s*CPS, min((s+1)*CPS, C)) and writes one FP64 partial per row
// block and column block.  NMAX bounds the column blocks a row block can
// need (ceil((M+1)/32)); instantiating no more keeps the accumulators, and
// so the registers, to what the lag range uses.
template <int ORD, int PATH, int WX, int NMAX>
__device__ __forceinline__ void moment_contract(C4Lds<PATH, WX> (&buf)[2],
                                                const float *__restrict__ xf,
                                                const uint4 *__restrict__ win4,
                                                const uint4 *__restrict__ win8h,
                                                const uint4 *__restrict__ win8l,
                                                double *__restrict__ part, int M, int P, int RB,
                                                int NCB, int64_t C, int CPS)
{
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, rl = lane & 31;
    const int rb = blockIdx.x * 4 + wave;
    const int s = blockIdx.y;
    const int64_t c0 = (int64_t)s * CPS;
    const int64_t c1 = c0 + CPS < C ? c0 + CPS : C;
    if (c0 >= c1)
        return;

    // this lane's row; column blocks = those of the workgroup's last row
    // (rows are ordered by their bound, so it has the largest)
    int a = 0, b = 0, c = 0, bound = 0;
    if (rb < RB && rb * 32 + rl < P)
        row_offsets<ORD>(M, rb * 32 + rl, a, b, c, bound);
    int last = blockIdx.x * 128 + 127;
    if (last > P - 1)
        last = P - 1;
    int al, bl, cl, boundl;
    row_offsets<ORD>(M, last, al, bl, cl, boundl);
    const int ncol = __builtin_amdgcn_readfirstlane(boundl / 32 + 1);
    switch (ncol) {
#define C4CASE(K)                                                                           \
    case K:                                                                                 \
        if constexpr (32 * K <= WX && K <= NMAX)                                            \
            c4_run<ORD, PATH, WX, K>(buf, xf, win4, win8h, win8l, part, a, b, c, rb, s,       \
                                     RB, NCB, c0, c1, wave, lane);                          \
        break;
        C4CASE(1) C4CASE(2) C4CASE(3) C4CASE(4)
#undef C4CASE
    default:
        break;
    }
}

// Up to two column blocks the accumulators and operands fit 256 registers:
// two workgroups per compute unit (two waves per SIMD) hide each other's
// latencies.
template <int PATH, int WX, int NMAX>
__global__ void __launch_bounds__(256, 1)
k_c4_contract(const float *__restrict__ xf, const uint4 *__restrict__ win4,
              const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l,
              double *__restrict__ part, int M, int P, int RB, int NCB, int64_t C, int CPS)
{
    __shared__ C4Lds<PATH, WX> buf[2];
    moment_contract<4, PATH, WX, NMAX>(buf, xf, win4, win8h, win8l, part, M, P, RB, NCB, C,
                                       CPS);
}

// Order five: rows (a, b, c), product row x_i x_{i+a} x_{i+b} x_{i+c}
// against the Hankel columns x_{i+d}, d <= c.
template <int PATH, int WX, int NMAX>
__global__ void __launch_bounds__(256, 1)
k_c5_contract(const float *__restrict__ xf, const uint4 *__restrict__ win4,
              const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l,
              double *__restrict__ part, int M, int P, int RB, int NCB, int64_t C, int CPS)
{
    __shared__ C4Lds<PATH, WX> buf[2];
    moment_contract<5, PATH, WX, NMAX>(buf, xf, win4, win8h, win8l, part, M, P, RB, NCB, C,
                                       CPS);
}

// Sum the S chunk-range partials of one (row block, column block) in a fixed
// order and scatter to mtab[r][d] (scaled sums, d <= the row's bound only).
// One thread per element: blockIdx.x = (row block, column block, quarter).
template <int ORD>
__device__ __forceinline__ void moment_reduce(const double *__restrict__ part, int M, int P,
                                              int RB, int NCB, int S, double *__restrict__ mtab)
{
    const int q = blockIdx.x & 3;
    const int rb = (blockIdx.x >> 2) / NCB, cb = (blockIdx.x >> 2) % NCB;
    int al, bl, cl, boundl;
    row_offsets<ORD>(M, (rb * 32 + 31 < P ? rb * 32 + 31 : P - 1), al, bl, cl, boundl);
    if (cb > boundl / 32)
        return;
    const int e = threadIdx.x + 256 * q;
    double sum = 0.0;
    // unrolled so the loads go out ahead; the adds keep their order
#pragma unroll 8
    for (int s = 0; s < S; ++s)
        sum += part[(((int64_t)s * RB + rb) * NCB + cb) * 1024 + e];
    const int v = e >> 6, lane = e & 63;
    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), col = lane & 31;
    const int r = rb * 32 + row, d = cb * 32 + col;
    if (r < P) {
        int a, b, c, bound;
        row_offsets<ORD>(M, r, a, b, c, bound);
        if (d <= bound)
            mtab[(int64_t)r * (M + 1) + d] = sum;
    }
}

__global__ void __launch_bounds__(256)
k_c4_reduce(const double *__restrict__ part, int M, int P, int RB, int NCB, int S,
            double *__restrict__ m4tab)
{
    moment_reduce<4>(part, M, P, RB, NCB, S, m4tab);
}

__global__ void __launch_bounds__(256)
k_c5_reduce(const double *__restrict__ part, int M, int P, int RB, int NCB, int S,
            double *__restrict__ m5tab)
{
    moment_reduce<5>(part, M, P, RB, NCB, S, m5tab);
}

// c2 partial sums sum_i x~_i x~_{i+d} (scaled by s^2), d = 0..M, FP64 from
// the input.
template <typename T>
__global__ void __launch_bounds__(256)
k_c2_dot(const T *__restrict__ x, int64_t n, const double *__restrict__ stats, int nblocks,
         double *__restrict__ dpart)
{
    __shared__ double red[256];
    const int d = blockIdx.x / nblocks, blk = blockIdx.x % nblocks;
    const double mu = stats[0], sc = stats[1];
    // four independent partial sums per thread (so the loads go out
    // together), combined in a fixed order
    const int64_t stride = (int64_t)nblocks * 256;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = (int64_t)blk * 256 + threadIdx.x;
    for (; i + 3 * stride + d < n; i += 4 * stride) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j = i + k * stride;
            a4[k] += (((double)x[j] - mu) * sc) * (((double)x[j + d] - mu) * sc);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t j = i + k * stride;
        if (j + d < n)
            a4[k] += (((double)x[j] - mu) * sc) * (((double)x[j + d] - mu) * sc);
    }
    red[threadIdx.x] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        dpart[blockIdx.x] = red[0];
}

// c2(d) = (sum of partials) / (n s^2), d = 0..M.
__global__ void __launch_bounds__(64)
k_c2_final(const double *__restrict__ dpart, int M, int nblocks, const double *__restrict__ stats,
           int64_t n, double *__restrict__ c2)
{
    const int d = blockIdx.x * 64 + threadIdx.x;
    if (d > M)
        return;
    double s = 0.0;
    // unrolled so the loads go out ahead; the adds keep their order
#pragma unroll 8
    for (int k = 0; k < nblocks; ++k)
        s += dpart[d * nblocks + k];
    const double sc = stats[1];
    c2[d] = s / ((double)n * sc * sc);
}

__global__ void __launch_bounds__(256)
k_c4_out(const double *__restrict__ m4tab, const double *__restrict__ c2,
         const double *__restrict__ stats, int M, double *__restrict__ out)
{
    const int side = 2 * M + 1;
    const int64_t tot = (int64_t)side * side * side;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot)
        return;
    const int t3 = (int)(idx % side) - M;
    const int t2 = (int)((idx / side) % side) - M;
    const int t1 = (int)(idx / ((int64_t)side * side)) - M;
    out[idx] = c4_at(m4tab, c2, M, stats[4], t1, t2, t3);
}

// Order five needs the third-order cumulants for its corrections: the FP64
// sums sum_i x~_i x~_{i+a} x~_{i+b} (scaled by s^3) over the pairs b <= a of
// F, from the input.  A workgroup takes C3D_BS samples (and the M after
// them) into LDS as FP64 x~ and strides over such blocks.  Thread t owns the
// lag a = t mod (M+1) and every (256 / (M+1))-th run of C3D_RUN samples: it
// forms the products x~_i x~_{i+a} of a run once and meets them with the
// window x~_{i+b}, b = 0..a, held in registers, keeping its a + 1 sums in
// registers too.  At the end the threads of one lag add their sums in slot
// order and each pair's workgroup partial goes to dpart[pair][workgroup]
// (fixed order throughout: the result is bitwise reproducible).
constexpr int C3D_RUN = 8;
constexpr int C3D_RED = 128 * (C5_MAX_M + 2);   // >= (256 / (M+1)) * pairs(M)

template <typename T>
__global__ void __launch_bounds__(256)
k_c3_dot(const T *__restrict__ x, int64_t n, const double *__restrict__ stats, int M,
         double *__restrict__ dpart)
{
    __shared__ double sx[C3D_BS + C5_MAX_M + C3D_RUN];
    __shared__ double red[C3D_RED];
    const int tid = threadIdx.x;
    const int L = M + 1, S = 256 / L, pairs = L * (L + 1) / 2;
    const int a = tid % L, slot = tid / L;
    const double mu = stats[0], sc = stats[1];
    double acc[C5_MAX_M + 1];
#pragma unroll
    for (int b = 0; b <= C5_MAX_M; ++b)
        acc[b] = 0.0;
    const int64_t nblk = (n + C3D_BS - 1) / C3D_BS;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t i0 = blk * C3D_BS;
        __syncthreads();   // every read of the previous block is done
        for (int j = tid; j < C3D_BS + M + C3D_RUN; j += 256) {
            const int64_t i = i0 + j;
            sx[j] = i < n ? ((double)x[i] - mu) * sc : 0.0;
        }
        __syncthreads();
        if (slot < S) {
            for (int r = slot; r < C3D_BS / C3D_RUN; r += S) {
                const int base = r * C3D_RUN;
                double v[C3D_RUN + C5_MAX_M];
#pragma unroll
                for (int k = 0; k < C3D_RUN + C5_MAX_M; ++k)
                    v[k] = k < C3D_RUN + M ? sx[base + k] : 0.0;
                double y[C3D_RUN];
#pragma unroll
                for (int j = 0; j < C3D_RUN; ++j)
                    y[j] = v[j] * sx[base + j + a];
#pragma unroll
                for (int b = 0; b <= C5_MAX_M; ++b)
                    if (b <= a) {
#pragma unroll
                        for (int j = 0; j < C3D_RUN; ++j)
                            acc[b] = fma(y[j], v[b + j], acc[b]);
                    }
            }
        }
    }
    __syncthreads();
    if (slot < S) {
#pragma unroll
        for (int b = 0; b <= C5_MAX_M; ++b)
            if (b <= a)
                red[slot * pairs + pair_offset(M, b) + (a - b)] = acc[b];
    }
    __syncthreads();
    for (int pr = tid; pr < pairs; pr += 256) {
        double s = 0.0;
        for (int k = 0; k < S; ++k)
            s += red[k * pairs + pr];
        dpart[(int64_t)pr * gridDim.x + blockIdx.x] = s;
    }
}

// c3tab[a][b] = (sum of partials) / (n s^3), b <= a (stride M + 1): one
// workgroup per pair, a fixed-order tree over its workgroup partials.
__global__ void __launch_bounds__(256)
k_c3_final(const double *__restrict__ dpart, int M, int nblocks,
           const double *__restrict__ stats, int64_t n, double *__restrict__ c3tab)
{
    __shared__ double red[256];
    const int pr = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 256)
        s += dpart[(int64_t)pr * nblocks + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int a, b;
        pair_ab(M, pr, a, b);
        const double sc = stats[1];
        c3tab[a * (M + 1) + b] = red[0] / ((double)n * sc * sc * sc);
    }
}

// The small tables every order-five output reads, staged in LDS once per
// workgroup: Parzen weights d(m) for |m| <= M (the values parzen_d gives),
// c2(0..M) and the third-order cumulants c3tab[a][b] (stride M + 1).
struct C5Tables {
    double d[2 * C5_MAX_M + 1];
    double c2[C5_MAX_M + 1];
    double c3[(C5_MAX_M + 1) * (C5_MAX_M + 1)];
};

__device__ inline void load_c5_tables(C5Tables &t, const double *__restrict__ c2,
                                      const double *__restrict__ c3tab, int M)
{
    for (int i = threadIdx.x; i <= 2 * M; i += blockDim.x)
        t.d[i] = parzen_d(i - M, M);
    for (int i = threadIdx.x; i <= M; i += blockDim.x)
        t.c2[i] = c2[i];
    for (int i = threadIdx.x; i < (M + 1) * (M + 1); i += blockDim.x)
        t.c3[i] = c3tab[i];
    __syncthreads();
}

// window5 from the staged Parzen weights (0 beyond |m| > M).
__device__ inline double window5_tab(const double *d, int t1, int t2, int t3, int t4, int M,
                                     int window)
{
    if (window == HOS_WIN_NONE)
        return 1.0;
    auto dv = [&](int m) { return (m < -M || m > M) ? 0.0 : d[m + M]; };
    double w = dv(t1) * dv(t2) * dv(t3) * dv(t4);
    if (window == HOS_WIN_PARZEN)
        w *= dv(t2 - t1) * dv(t3 - t1) * dv(t4 - t1) * dv(t3 - t2) * dv(t4 - t2) * dv(t4 - t3);
    return w;
}

// Both kernels stride over their outputs from a bounded grid, so each
// workgroup stages the tables once for many outputs; indices fit 32 bits
// ((2M+1)^4 <= 81^4 and N^4 <= 96^4).
__global__ void __launch_bounds__(256)
k_c5_out(const double *__restrict__ m5tab, const double *__restrict__ c2,
         const double *__restrict__ c3tab, const double *__restrict__ stats, int M,
         double *__restrict__ out)
{
    __shared__ C5Tables tab;
    load_c5_tables(tab, c2, c3tab, M);
    const uint32_t side = 2 * M + 1, tot = side * side * side * side;
    const double norm5 = stats[4] * stats[1];
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += gridDim.x * blockDim.x) {
        uint32_t r = idx;
        const int t4 = (int)(r % side) - M;
        r /= side;
        const int t3 = (int)(r % side) - M;
        r /= side;
        const int t2 = (int)(r % side) - M;
        const int t1 = (int)(r / side) - M;
        out[idx] = c5_at(m5tab, tab.c2, tab.c3, M, norm5, t1, t2, t3, t4);
    }
}

// The windowed c5 folded onto the N^4 DFT grid (index w mod N, aliases
// summed; c5 read from the (2M+1)^4 cube k_c5_out wrote, whose zeros
// beyond span M lie where the window vanishes anyway) and transformed
// along the last axis in LDS: a workgroup takes
// CBP pairs of lines L = (m1 N + m2) N + m3, the two real lines of a pair
// travel as one complex sequence Z (lines L and L + 1 as its real and
// imaginary parts), and after the DFT
//   X_L(k) = (Z(k) + conj Z(N-k)) / 2,  X_{L+1}(k) = (Z(k) - conj Z(N-k)) / 2i
// go to Q; the three other axes follow (launch_fft4_tail).
constexpr int C5L_LDS = 2048;   // complex values of the line buffer

__global__ void __launch_bounds__(256)
k_c5_lines(const double *__restrict__ c5, int M, const double2 *__restrict__ tw, FftRadices fr,
           int CBP, int window, double2 *__restrict__ Q)
{
    __shared__ double2 sm[C5L_LDS];
    __shared__ double dwin[2 * C5_MAX_M + 1];
    for (int i = threadIdx.x; i <= 2 * M; i += blockDim.x)
        dwin[i] = parzen_d(i - M, M);
    __syncthreads();
    const int N = fr.n;
    const uint32_t lines = (uint32_t)N * N * N;
    const uint32_t side = 2 * M + 1;
    // the ten-difference Parzen product (the only window the spectra take)
    // vanishes once the span of {0, w1, .., w4} reaches M (d(m) = 0 from
    // |m| = M on; at M = 0 from |m| = 1): such lags are skipped before any
    // factor is formed, whole lines (the span of {0, w1, w2, w3}) at once
    const int zspan = M > 0 ? M : 1;
    auto fold = [&](uint32_t L, int m4) {
        double sum = 0.0;
        if (L >= lines)
            return sum;
        const int m3 = (int)(L % N), m2 = (int)((L / N) % N), m1 = (int)(L / ((uint32_t)N * N));
        for (int w1 = m1 - N; w1 <= m1; w1 += N) {
            if (w1 < -M || w1 > M)
                continue;
            for (int w2 = m2 - N; w2 <= m2; w2 += N) {
                if (w2 < -M || w2 > M)
                    continue;
                for (int w3 = m3 - N; w3 <= m3; w3 += N) {
                    if (w3 < -M || w3 > M)
                        continue;
                    const int lo3 = min(min(0, w1), min(w2, w3)),
                              hi3 = max(max(0, w1), max(w2, w3));
                    if (window == HOS_WIN_PARZEN && hi3 - lo3 >= zspan)
                        continue;
                    const uint32_t row =
                        (((uint32_t)(w1 + M) * side + (uint32_t)(w2 + M)) * side +
                         (uint32_t)(w3 + M)) * side;
                    for (int w4 = m4 - N; w4 <= m4; w4 += N) {
                        if (w4 < -M || w4 > M)
                            continue;
                        if (window == HOS_WIN_PARZEN &&
                            max(hi3, w4) - min(lo3, w4) >= zspan)
                            continue;
                        const double wv = window5_tab(dwin, w1, w2, w3, w4, M, window);
                        if (wv != 0.0)
                            sum += wv * c5[row + (uint32_t)(w4 + M)];
                    }
                }
            }
        }
        return sum;
    };
    const uint32_t L0 = blockIdx.x * 2u * (uint32_t)CBP;
    for (int e = threadIdx.x; e < CBP * N; e += 256) {
        const int p = e / N, m4 = e - p * N;
        sm[e] = make_double2(fold(L0 + 2 * p, m4), fold(L0 + 2 * p + 1, m4));
    }
    __syncthreads();
    fft_lds<256, C5L_LDS>(sm, tw, fr, CBP);
    for (int e = threadIdx.x; e < CBP * N; e += 256) {
        const int p = e / N, k = e - p * N;
        const uint32_t L = L0 + 2 * p;
        const double2 z = sm[p * N + k], zc = sm[p * N + (k == 0 ? 0 : N - k)];
        if (L < lines)
            Q[(int64_t)L * N + k] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        if (L + 1 < lines)
            Q[(int64_t)(L + 1) * N + k] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
}

template <int PATH, int WX, int NMAX>
void launch_c4_t(const C4Plan &p, char *ws, hipStream_t s)
{
    dim3 grid((p.RB + 3) / 4, p.S);
    k_c4_contract<PATH, WX, NMAX><<<grid, 256, 0, s>>>(
        (const float *)(ws + p.off_xf), (const uint4 *)(ws + p.off_win4),
        (const uint4 *)(ws + p.off_win8h), (const uint4 *)(ws + p.off_win8l),
        (double *)(ws + p.off_part), p.M, p.P, p.RB, p.NCB, p.C, p.CPS);
}

template <int PATH, int WX, int NMAX>
void launch_c5_t(const C4Plan &p, char *ws, hipStream_t s)
{
    dim3 grid((p.RB + 3) / 4, p.S);
    k_c5_contract<PATH, WX, NMAX><<<grid, 256, 0, s>>>(
        (const float *)(ws + p.off_xf), (const uint4 *)(ws + p.off_win4),
        (const uint4 *)(ws + p.off_win8h), (const uint4 *)(ws + p.off_win8l),
        (double *)(ws + p.off_part), p.M, p.P, p.RB, p.NCB, p.C, p.CPS);
}

template <int WX, int NMAX>
void launch_c4_path(const C4Plan &p, char *ws, hipStream_t s)
{
    if (p.ord == 5) {
        if (p.path == HOS_PATH_FP32)
            launch_c5_t<HOS_PATH_FP32, WX, NMAX>(p, ws, s);
        else if (p.path == HOS_PATH_SPLIT_FP16)
            launch_c5_t<HOS_PATH_SPLIT_FP16, WX, NMAX>(p, ws, s);
        else
            launch_c5_t<HOS_PATH_SPLIT_BF16, WX, NMAX>(p, ws, s);
        return;
    }
    if (p.path == HOS_PATH_FP32)
        launch_c4_t<HOS_PATH_FP32, WX, NMAX>(p, ws, s);
    else if (p.path == HOS_PATH_SPLIT_FP16)
        launch_c4_t<HOS_PATH_SPLIT_FP16, WX, NMAX>(p, ws, s);
    else
        launch_c4_t<HOS_PATH_SPLIT_BF16, WX, NMAX>(p, ws, s);
}

}  // namespace

int c4_window_entries(int M)
{
    // the staged window must reach x_{i+a}, x_{i+b} (+7) and the Hankel
    // columns 32 NCB - 1 (+7) past the chunk's last group: one of 64/128/192
    const int ncb = (M + 1 + 31) / 32;
    const int need = 32 * ncb + 16;
    if (need <= 64)
        return 64;
    if (need <= 128)
        return 128;
    return 192;
}

hipError_t launch_c4_contract(const C4Plan &p, char *ws, hipStream_t s)
{
    // the window (WX) and the largest column-block count (NCB) of the lag
    // range: WX 64 holds one block, 128 two or three, 192 four
    if (p.WX == 64)
        launch_c4_path<64, 1>(p, ws, s);
    else if (p.WX == 128 && p.NCB <= 2)
        launch_c4_path<128, 2>(p, ws, s);
    else if (p.WX == 128)
        launch_c4_path<128, 3>(p, ws, s);
    else
        launch_c4_path<192, 4>(p, ws, s);
    return hipGetLastError();
}

hipError_t launch_c4_reduce(const void *x, int dtype, const C4Plan &p, char *ws, hipStream_t s)
{
    if (p.ord == 5)
        k_c5_reduce<<<p.RB * p.NCB * 4, 256, 0, s>>>((const double *)(ws + p.off_part), p.M, p.P,
                                                     p.RB, p.NCB, p.S, (double *)(ws + p.off_m4));
    else
        k_c4_reduce<<<p.RB * p.NCB * 4, 256, 0, s>>>((const double *)(ws + p.off_part), p.M, p.P,
                                                     p.RB, p.NCB, p.S, (double *)(ws + p.off_m4));
    const double *stats = (const double *)(ws + p.off_stats);
    double *dpart = (double *)(ws + p.off_c2part);
    const int grid = (p.M + 1) * p.dot_blocks;
    if (dtype == HOS_F64)
        k_c2_dot<double><<<grid, 256, 0, s>>>((const double *)x, p.n, stats, p.dot_blocks, dpart);
    else
        k_c2_dot<float><<<grid, 256, 0, s>>>((const float *)x, p.n, stats, p.dot_blocks, dpart);
    k_c2_final<<<(p.M + 64) / 64, 64, 0, s>>>(dpart, p.M, p.dot_blocks, stats, p.n,
                                              (double *)(ws + p.off_c2));
    if (p.ord == 5) {
        const int pairs = (p.M + 1) * (p.M + 2) / 2;
        double *c3part = (double *)(ws + p.off_c3part);
        if (dtype == HOS_F64)
            k_c3_dot<double><<<p.c3_blocks, 256, 0, s>>>((const double *)x, p.n, stats, p.M,
                                                         c3part);
        else
            k_c3_dot<float><<<p.c3_blocks, 256, 0, s>>>((const float *)x, p.n, stats, p.M,
                                                        c3part);
        k_c3_final<<<pairs, 256, 0, s>>>(c3part, p.M, p.c3_blocks, stats, p.n,
                                          (double *)(ws + p.off_c3tab));
    }
    return hipGetLastError();
}

hipError_t launch_c5_finish(const C4Plan &p, int window, int nfft, double *c5, double *Q,
                            char *ws, hipStream_t s)
{
    const double *m5 = (const double *)(ws + p.off_m4);
    const double *c2 = (const double *)(ws + p.off_c2);
    const double *c3 = (const double *)(ws + p.off_c3tab);
    const double *stats = (const double *)(ws + p.off_stats);
    // bounded grids: 8 workgroups per CU, each striding over its outputs
    const int64_t gmax = 8 * 256;
    // the spectrum folds the cumulant cube: the caller's c5, or a workspace
    // copy when only Q is asked for
    double *cube = c5 ? c5 : (Q ? (double *)(ws + p.off_cube) : nullptr);
    if (cube) {
        const int64_t side = 2 * p.M + 1, tot = side * side * side * side;
        const int64_t grid = std::min<int64_t>((tot + 255) / 256, gmax);
        k_c5_out<<<(unsigned)grid, 256, 0, s>>>(m5, c2, c3, stats, p.M, cube);
    }
    if (Q) {   // fold, window and the transforms along the last axis
        const FftRadices fr = factor(nfft);
        const int64_t lines = (int64_t)nfft * nfft * nfft;
        const int CBP = std::min(32, C5L_LDS / nfft);
        const int64_t grid = (lines + 2 * CBP - 1) / (2 * CBP);
        k_c5_lines<<<(unsigned)grid, 256, 0, s>>>(cube, p.M, (const double2 *)(ws + p.off_twid),
                                                  fr, CBP, window, (double2 *)Q);
    }
    return hipGetLastError();
}

hipError_t launch_c4_finish(const C4Plan &p, int window, int nfft, double *c4, double *T,
                            char *ws, hipStream_t s)
{
    const double *m4 = (const double *)(ws + p.off_m4);
    const double *c2 = (const double *)(ws + p.off_c2);
    const double *stats = (const double *)(ws + p.off_stats);
    // the spectrum folds the cumulant cube: the caller's c4, or a workspace
    // copy when only T is asked for
    double *cube = c4 ? c4 : (T ? (double *)(ws + p.off_cube) : nullptr);
    if (cube) {
        const int64_t side = 2 * p.M + 1, tot = side * side * side;
        k_c4_out<<<(tot + 255) / 256, 256, 0, s>>>(m4, c2, stats, p.M, cube);
    }
    if (T) {   // fold + window + the m3 transforms (k_fft.hip); k2 and k1 follow
        hipError_t e = launch_tri_lines(cube, p.M, nfft, window,
                                        (const double2 *)(ws + p.off_twid), T, s);
        if (e != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

}  // namespace hos
