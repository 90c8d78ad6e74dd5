// k_adjoint.hip -- gradient of the bispectrum-matching loss with respect to
// the input series (the adjoint of the estimator), recomputing the product
// terms from the series instead of storing anything of the forward pass.
//
// Loss: L = sum_k |B(k) - T(k)|^2 over the principal domain, B the windowed
// DFT of c3 (the part DFT and raw bispectrum of Algorithm DBS for the sign and the domain).  With
// R = B - T, the weight of each lag is
//     G(w) = dL/dc3(w) = 2 W3(w) Re sum_k R_k e^{+2 pi i <k,w>/N},
// obtained as the real part of a forward DFT of conj(2 R) placed on the
// grid.  Differentiating c3(w) = (1/n) sum_t x_t x_{t+w1} x_{t+w2} gives,
// for the mean-removed series x,
//     g_j = dL/dx_j = sum_{u,v} K(u,v) x_{j+u} x_{j+v},
//     K(u,v) = (1/n) [G(u,v) + G(-u, v-u) + G(v-u, -u)],
// a quadratic form of the (2M+1)-sample window around j (K vanishes
// outside the hexagon |u|,|v|,|u-v| <= M).  Only the symmetric part of K
// matters; it is stored block-upper-triangular (32 x 32 blocks: diagonal
// blocks once, blocks above twice, below none), so
//     g_j = sum_u x_{j+u} Z[j][u],   Z[j][u] = sum_v K2(u,v) x_{j+v}:
// a matrix-core contraction of the Hankel matrix H[j][v] = x_{j+v} with K2,
// followed by a row-wise dot product with the same Hankel rows.  The mean
// removal contributes dL/dx_j = g_j - mean(g).
#include "hos_internal.h"
#include "hos_device.h"

namespace hos {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


// Packed index of (k1, k2) in the principal domain 0 <= k2 <= k1,
// k1 + k2 <= H = floor((N-1)/2), or -1.  Row k1 holds min(k1, H - k1) + 1
// points: k1 + 1 up to h = floor(H/2), H - k1 + 1 after.
__device__ inline int pd_index(int k1, int k2, int N)
{
    const int H = (N - 1) / 2;
    if (k2 > k1 || k1 + k2 > H)
        return -1;
    const int h = H / 2, p = k1 < h + 1 ? k1 : h + 1;
    int start = p * (p + 1) / 2;
    if (k1 > h + 1)
        start += (k1 - h - 1) * (H + 1) - ((k1 - 1) * k1 / 2 - h * (h + 1) / 2);
    return start + k2;
}

// The bits of max |K2| (slot 6 of a series' statistics) accumulate by an
// atomic maximum over non-negative doubles, whose order is that of their
// bit patterns: the result does not depend on the order of the updates.
__device__ inline unsigned long long *kmax_bits(const SeriesDesc &d, char *ws)
{
    return (unsigned long long *)((double *)(ws + d.ws_off + d.o_stats) + 6);
}

// grid = conj(2 dL (B - T)) on the principal domain, 0 elsewhere; also
// clears the running max |K2| that k_adj_kbuild fills.
__global__ void __launch_bounds__(256)
k_adj_resid(const SeriesDesc *__restrict__ sd, const double2 *__restrict__ B_pd,
            const double2 *__restrict__ target, const double *__restrict__ dL,
            char *__restrict__ ws)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int N = d.N, H = (N - 1) / 2, C2 = H / 2 + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0)
        *kmax_bits(d, ws) = 0ull;
    // the corner k1 <= H, k2 <= H / 2 holds the principal domain; the DFT
    // reads nothing outside it
    if (idx >= (int64_t)(H + 1) * C2)
        return;
    const int k1 = (int)(idx / C2), k2 = (int)(idx % C2);
    const int p = pd_index(k1, k2, N);
    double2 v = make_double2(0.0, 0.0);
    if (p >= 0) {
        const double2 b = B_pd[d.pd_off + p], t = target[p];
        const double c = 2.0 * dL[0];
        v = make_double2(c * (b.x - t.x), -c * (b.y - t.y));
    }
    ((double2 *)(ws + d.grid_off))[(int64_t)k1 * N + k2] = v;
}

// K2 in FP64 over the 32-blocks on and above the block diagonal of
// [0, KP)^2 (u' = u + M, v' = v + M; padding is 0; the blocks below are
// never read, so they are not written), and the running max |K2| (a
// workgroup's maximum, then one atomic maximum).  One workgroup per block
// (bu, bv), bv >= bu; thread t holds row u' = 32 bu + t / 8 and the four
// columns v' = 32 bv + 4 (t mod 8) + j.  Of the six terms of
// K(u,v) + K(v,u) = G(u,v) + G(-u,v-u) + G(v-u,-u) + G(v,u) + G(-v,u-v) + G(u-v,-v)
// the first two run along rows of G as v runs and are read directly; the
// other four would run down columns or diagonals, so each is first staged
// in LDS as the rectangle of G rows it touches (at most 63 x 32), read
// along rows.
constexpr int KB_LD = 33;   // LDS row pitch (doubles) of a staged rectangle

__global__ void __launch_bounds__(256)
k_adj_kbuild(const SeriesDesc *__restrict__ sd, char *__restrict__ ws)
{
    __shared__ double buf[64 * KB_LD];
    __shared__ double red[4];
    const SeriesDesc &d = sd[blockIdx.y];
    const int KP = d.KP, M = d.M, S = 2 * M + 1, NB = KP >> 5;
    // block number -> (bu, bv), bv >= bu, row-major over the upper triangle
    int t = blockIdx.x, bu = 0;
    while (bu < NB && t >= NB - bu) {
        t -= NB - bu;
        ++bu;
    }
    if (bu >= NB)
        return;   // beyond this series' blocks (uniform over the workgroup)
    const int bv = bu + t;
    const double *Gt = (const double *)(ws + d.ws_off + d.o_gtab);
    auto G = [&](int a, int b) {
        return (a < -M || a > M || b < -M || b > M) ? 0.0 : Gt[(int64_t)(a + M) * S + (b + M)];
    };
    const int tid = threadIdx.x;
    const int iu = tid >> 3, jv = 4 * (tid & 7);
    const int u0 = 32 * bu - M, v0 = 32 * bv - M;
    const int u = u0 + iu;
    double acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + jv + j;
        acc[j] = G(u, v) + G(-u, v - u);
    }
    // stage the rectangle rows [r0, r0 + nr) x columns [c0, c0 + 32) of G,
    // then add buf[row(j) - r0][col(j) - c0] to acc[j]
    auto stage = [&](int r0, int nr, int c0) {
        __syncthreads();
        for (int e = tid; e < nr * 32; e += 256) {
            const int rr = e >> 5, cc = e & 31;
            buf[rr * KB_LD + cc] = G(r0 + rr, c0 + cc);
        }
        __syncthreads();
    };
    // G(v - u, -u): rows v - u in [v0 - u0 - 31, v0 - u0 + 31], columns -u
    stage(v0 - u0 - 31, 63, -u0 - 31);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + jv + j;
        acc[j] += buf[(v - u - (v0 - u0 - 31)) * KB_LD + (-u - (-u0 - 31))];
    }
    // G(v, u): rows v in [v0, v0 + 32), columns u
    stage(v0, 32, u0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        acc[j] += buf[(jv + j) * KB_LD + iu];
    // G(u - v, -v): rows u - v in [u0 - v0 - 31, u0 - v0 + 31], columns -v
    stage(u0 - v0 - 31, 63, -v0 - 31);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + jv + j;
        acc[j] += buf[(u - v - (u0 - v0 - 31)) * KB_LD + (-v - (-v0 - 31))];
    }
    // G(-v, u - v): rows -v in [-v0 - 31, -v0], columns u - v in
    // [u0 - v0 - 31, u0 - v0 + 31]: staged transposed (row = column offset)
    __syncthreads();
    for (int e = tid; e < 32 * 63; e += 256) {
        // consecutive threads read consecutive columns of one row of G
        const int rr = e / 63, cc = e - rr * 63;   // rr: -v offset, cc: u - v offset
        buf[cc * KB_LD + rr] = G(-v0 - 31 + rr, u0 - v0 - 31 + cc);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + jv + j;
        acc[j] += buf[(u - v - (u0 - v0 - 31)) * KB_LD + (-v - (-v0 - 31))];
    }
    const int up = 32 * bu + iu;
    double m = 0.0;
    double *K64 = (double *)(ws + d.ws_off + d.o_k64);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int vp = 32 * bv + jv + j;
        double val = 0.0;
        if (up <= 2 * M && vp <= 2 * M) {
            const double ks = 0.5 * acc[j] / (double)d.n;
            val = bv > bu ? 2.0 * ks : ks;
        }
        K64[(int64_t)up * KP + vp] = val;
        m = fmax(m, fabs(val));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        m = fmax(m, __shfl_xor(m, off, 64));
    if ((tid & 63) == 0)
        red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(kmax_bits(d, ws), (unsigned long long)__double_as_longlong(m));
    }
}

// Power-of-two scale sk with max|K2| sk in [2^14, 2^15) (1 when K2 is 0 or
// not finite).
__device__ inline double kscale(double mx)
{
    double sk = 1.0;
    if (mx > 0.0 && isfinite(mx)) {
        int e;
        frexp(mx, &e);
        sk = ldexp(1.0, 15 - e);
    }
    return sk;
}

// K2 sk rounded for the matrix cores: FP32, or hi + lo halves.
template <int PATH>
__global__ void __launch_bounds__(256)
k_adj_ksplit(const SeriesDesc *__restrict__ sd, char *__restrict__ ws)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d.KP * d.KP)
        return;
    char *r = ws + d.ws_off;
    // idx enumerates the stored order: k_adj_contract's B fragments, one per
    // (32-block U of u, 32-block V of v, 16-wide k-group g), each 64 lanes x
    // 8 consecutive v of one row u (lane = u mod 32 + 32 h, v = 32V + 16g +
    // 8h + e), so that a wave's fragment load is one contiguous run
    const int NU = d.KP >> 5;
    const int e = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
    const int64_t f = idx >> 9;
    const int g = (int)(f & 1), V = (int)((f >> 1) % NU), U = (int)((f >> 1) / NU);
    if (V < U)
        return;   // below the block diagonal: never read
    const int u = U * 32 + (lane & 31), vv = V * 32 + 16 * g + 8 * (lane >> 5) + e;
    // rows of odd 32-blocks of u are stored negated (see k_adj_contract)
    const double sk = kscale(__longlong_as_double((long long)*kmax_bits(d, ws)));
    if (idx == 0)
        ((double *)(r + d.o_stats))[5] = sk;   // for k_adj_final
    const double sg = (U & 1) ? -1.0 : 1.0;
    const float v = (float)(((const double *)(r + d.o_k64))[(int64_t)u * d.KP + vv] * sk * sg);
    if constexpr (PATH == HOS_PATH_FP32) {
        ((float *)(r + d.o_kh))[idx] = v;
    } else if constexpr (PATH == HOS_PATH_SPLIT_FP16) {
        const _Float16 hi = (_Float16)v;
        const _Float16 lo = (_Float16)(v - (float)hi);
        ((_Float16 *)(r + d.o_kh))[idx] = hi;
        ((_Float16 *)(r + d.o_kl))[idx] = lo;
    } else {
        const __bf16 hi = (__bf16)v;
        const __bf16 lo = (__bf16)(v - (float)hi);
        ((__bf16 *)(r + d.o_kh))[idx] = hi;
        ((__bf16 *)(r + d.o_kl))[idx] = lo;
    }
}

template <int PATH>
__device__ inline floatx16 mma16(uint4 a, uint4 b, floatx16 c)
{
    if constexpr (PATH == HOS_PATH_SPLIT_FP16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                      __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// g_j s^2 sk for ADJ_ROWS rows j per workgroup (blockIdx.y = series).  The
// workgroup stages the table entries its rows touch, [j0 - M, j0 + ADJ_ROWS
// + KP - M), in LDS; wave w owns rows j0 + 32 ADJ_NRB w + [0, 32 ADJ_NRB) as
// ADJ_NRB blocks of 32.  For each 32-block U of u it accumulates the
// transposed product Z^T = K2 H^T over the v blocks V >= U within the
// hexagon's reach (A = the K2 fragments from global memory, B = Hankel
// columns x_{j+v} from LDS; the first block starts the accumulators from
// zero inside the matrix-core op).  In that orientation a lane's column is
// one row j and its 16 values are 16 of the u, so the fold
// g_j += sum_u x_{j+u} Z[j][u] stays inside the lane: one FP64 multiply-add
// per value into a per-block partial (x in FP64 from LDS, the FP32 x FP32
// product exact in FP64), one FP64 partial per row block per lane, and the
// two lanes of a row are added at the end.
template <int PATH>
__global__ void __launch_bounds__(256, 2)
k_adj_contract(const SeriesDesc *__restrict__ sd, char *__restrict__ ws, int WA)
{
    constexpr int NRB = ADJ_NRB;
    extern __shared__ uint4 lds[];
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t j0 = (int64_t)blockIdx.x * ADJ_ROWS;
    if (j0 >= d.n)
        return;
    const int M = d.M, KP = d.KP, NU = KP >> 5, reach = (M + 31) >> 5;
    char *r = ws + d.ws_off;
    constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    // split paths: hi | lo window tables and the FP64 pairs; FP32: the FP32
    // window table and the FP64 pairs (WA entries each)
    float4 *s_f4 = (float4 *)lds;
    uint4 *s_h = lds, *s_l = lds + WA;
    double2 *s_d2 = (double2 *)(lds + (SPLIT ? 2 : 1) * WA);
    {
        // this series' window (WA is the largest over the batch)
        const int WAs = ADJ_ROWS + KP;
        const int64_t g0 = j0 - M;
        const float *xf = (const float *)(r + d.o_xf);
        if constexpr (SPLIT) {
            const uint4 *h = (const uint4 *)(r + d.o_win8h), *l = (const uint4 *)(r + d.o_win8l);
            for (int e = threadIdx.x; e < WAs; e += 256) {
                s_h[e] = h[g0 + e];
                s_l[e] = l[g0 + e];
            }
        } else {
            const float4 *f4 = (const float4 *)(r + d.o_win4);
            for (int e = threadIdx.x; e < WAs; e += 256)
                s_f4[e] = f4[g0 + e];
        }
        // entry e = (x_{g0+e}, x_{g0+e+1}) in FP64
        for (int e = threadIdx.x; e < WAs; e += 256)
            s_d2[e] = make_double2((double)xf[g0 + e], (double)xf[g0 + e + 1]);
    }
    __syncthreads();

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, rl = lane & 31, h = lane >> 5;
    const int jw = wave * 32 * NRB + rl;   // this lane's row j - j0 in block 0
    double E[NRB];
#pragma unroll
    for (int b = 0; b < NRB; ++b)
        E[b] = 0.0;
    // A fragments as k_adj_ksplit stores them: fragment (U, V, g) holds
    // lane l's 8 values at [(frag * 64 + l) * 8, + 8)
    const uint4 *kh = (const uint4 *)(r + d.o_kh), *kl = (const uint4 *)(r + d.o_kl);
    const floatx16 zero = {};
    for (int U = 0; U < NU; ++U) {
        floatx16 a[NRB];
        const int Vmax = min(NU - 1, U + reach);
        // one v block: 2 k-groups of 16
        auto vstep = [&](int V, bool first) __attribute__((always_inline)) {
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int vl = V * 32 + 16 * g + 8 * h;   // first v of this lane's 8
                const bool z = first && g == 0;
                const int64_t fl = ((int64_t)(U * NU + V) * 2 + g) * 64 + lane;
                if constexpr (SPLIT) {
                    const uint4 kH = kh[fl], kL = kl[fl];
#pragma unroll
                    for (int b = 0; b < NRB; ++b) {
                        const uint4 xh = s_h[jw + 32 * b + vl], xl = s_l[jw + 32 * b + vl];
                        a[b] = mma16<PATH>(kH, xh, z ? zero : a[b]);
                        a[b] = mma16<PATH>(kL, xh, a[b]);
                        a[b] = mma16<PATH>(kH, xl, a[b]);
                    }
                } else {
                    const float4 *kf = (const float4 *)(r + d.o_kh);
                    const float4 b0 = kf[2 * fl], b1 = kf[2 * fl + 1];
                    const float kk[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                    for (int b = 0; b < NRB; ++b) {
                        const float4 x0 = s_f4[jw + 32 * b + vl], x1 = s_f4[jw + 32 * b + vl + 4];
                        const float xx[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            a[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                kk[e], xx[e], z && e == 0 ? zero : a[b], 0, 0, 0);
                    }
                }
            }
        };
        vstep(U, true);
        for (int V = U + 1; V <= Vmax; ++V)
            vstep(V, false);
        // fold: value v of a lane is u = 32U + 8(v/4) + 4h + v%4 of its row
        // j.  Odd U ran on negated K2 rows, so the matrix cores' rounding
        // bias (toward -infinity) alternates in sign between blocks and
        // cancels; the sign is undone on the block's partial (exact).
        const double sg = (U & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int b = 0; b < NRB; ++b) {
            double part = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = jw + 32 * b + 32 * U + 8 * q + 4 * h;
                const double2 y01 = s_d2[o], y23 = s_d2[o + 2];
                part = __builtin_fma((double)a[b][4 * q + 0], y01.x, part);
                part = __builtin_fma((double)a[b][4 * q + 1], y01.y, part);
                part = __builtin_fma((double)a[b][4 * q + 2], y23.x, part);
                part = __builtin_fma((double)a[b][4 * q + 3], y23.y, part);
            }
            E[b] = __builtin_fma(sg, part, E[b]);
        }
    }
    // the two lanes of a row (h = 0, 1) hold disjoint u
    double *gt = (double *)(r + d.o_gtil);
#pragma unroll
    for (int b = 0; b < NRB; ++b) {
        const double t = E[b] + __shfl_xor(E[b], 32, 64);
        const int64_t j = j0 + jw + 32 * b;
        if (h == 0 && j < d.n)
            gt[j] = t;
    }
}

// dx_j = (g_j - mean g) / (s^2 sk), mean in a fixed order.
// Block sums of g~ for the mean: workgroup (b, series) adds the samples
// [b L, (b + 1) L) (L = ADJ_MEAN_BLOCK) by a fixed tree.

__global__ void __launch_bounds__(256)
k_adj_msum(const SeriesDesc *__restrict__ sd, char *__restrict__ ws)
{
    __shared__ double red[256];
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t j0 = (int64_t)blockIdx.x * ADJ_MEAN_BLOCK;
    if (j0 >= d.n)
        return;
    const char *r = ws + d.ws_off;
    const double *gt = (const double *)(r + d.o_gtil);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < ADJ_MEAN_BLOCK / 256; ++q) {
        const int64_t j = j0 + threadIdx.x + 256 * q;
        s += j < d.n ? gt[j] : 0.0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        ((double *)(ws + d.ws_off + d.o_msum))[blockIdx.x] = red[0];
}

// dx_j = (g_j - mean g) / (s^2 sk): the mean from the block sums added in
// block order, then workgroup (b, series) writes block b.
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_final(const SeriesDesc *__restrict__ sd, const char *__restrict__ ws, T *__restrict__ dx)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t j0 = (int64_t)blockIdx.x * ADJ_MEAN_BLOCK;
    if (j0 >= d.n)
        return;
    const char *r = ws + d.ws_off;
    const double *gt = (const double *)(r + d.o_gtil);
    const double *bs = (const double *)(r + d.o_msum);
    const double *stats = (const double *)(r + d.o_stats);
    const int nb = (int)((d.n + ADJ_MEAN_BLOCK - 1) / ADJ_MEAN_BLOCK);
    double sum = 0.0;
    for (int b = 0; b < nb; ++b)
        sum += bs[b];
    const double mean = sum / (double)d.n;
    const double inv = 1.0 / (stats[1] * stats[1] * stats[5]);
#pragma unroll
    for (int q = 0; q < ADJ_MEAN_BLOCK / 256; ++q) {
        const int64_t j = j0 + threadIdx.x + 256 * q;
        if (j < d.n)
            dx[d.x_off + j] = (T)((gt[j] - mean) * inv);
    }
}

template <int PATH>
void launch_adj_contract(const BatchHeader &h, const SeriesDesc *sd, char *ws, hipStream_t s)
{
    const int WA = (int)(ADJ_ROWS + h.max_KP);
    const size_t lds = (size_t)WA * 16 * (PATH == HOS_PATH_FP32 ? 2 : 3);
    const dim3 grid((unsigned)((h.max_n + ADJ_ROWS - 1) / ADJ_ROWS), (unsigned)h.batch);
    k_adj_contract<PATH><<<grid, 256, lds, s>>>(sd, ws, WA);
}

}  // namespace

hipError_t launch_batch_adjoint(const void *x, int dtype, const BatchHeader &h, const char *dplan,
                                int window, const double *B_pd, const double *target,
                                const double *dL, void *dx, char *ws, hipStream_t s)
{
    (void)x;
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    const int B = (int)h.batch;
    const int64_t Hm = (h.max_N - 1) / 2, corner = (Hm + 1) * (Hm / 2 + 1);
    k_adj_resid<<<dim3((unsigned)((corner + 255) / 256), B), 256, 0, s>>>(
        sd, (const double2 *)B_pd, (const double2 *)target, dL, ws);
    const FftGroup *groups = (const FftGroup *)((const char *)&h + h.groups_off);
    const int32_t *gser = (const int32_t *)(dplan + h.gseries_off);
    for (int g = 0; g < (int)h.n_groups; ++g) {
        const FftGroup &gr = groups[g];
        hipError_t e = launch_twiddles((double2 *)(ws + gr.twid_off), gr.N, s);
        // the residual's 2-D DFT, whose second pass writes the lag weights
        if (e == hipSuccess)
            e = launch_adj_gweights(gr, sd, gser, window, ws, s);
        if (e != hipSuccess)
            return e;
    }
    const int64_t k2 = h.max_KP * h.max_KP;
    const int64_t nbk = h.max_KP / 32;
    k_adj_kbuild<<<dim3((unsigned)(nbk * (nbk + 1) / 2), B), 256, 0, s>>>(sd, ws);
    const dim3 gk((unsigned)((k2 + 255) / 256), B);
    if (h.path == HOS_PATH_FP32) {
        k_adj_ksplit<HOS_PATH_FP32><<<gk, 256, 0, s>>>(sd, ws);
        launch_adj_contract<HOS_PATH_FP32>(h, sd, ws, s);
    } else if (h.path == HOS_PATH_SPLIT_FP16) {
        k_adj_ksplit<HOS_PATH_SPLIT_FP16><<<gk, 256, 0, s>>>(sd, ws);
        launch_adj_contract<HOS_PATH_SPLIT_FP16>(h, sd, ws, s);
    } else {
        k_adj_ksplit<HOS_PATH_SPLIT_BF16><<<gk, 256, 0, s>>>(sd, ws);
        launch_adj_contract<HOS_PATH_SPLIT_BF16>(h, sd, ws, s);
    }
    const dim3 gm((unsigned)((h.max_n + ADJ_MEAN_BLOCK - 1) / ADJ_MEAN_BLOCK), (unsigned)B);
    k_adj_msum<<<gm, 256, 0, s>>>(sd, ws);
    if (dtype == HOS_F64)
        k_adj_final<double><<<gm, 256, 0, s>>>(sd, ws, (double *)dx);
    else
        k_adj_final<float><<<gm, 256, 0, s>>>(sd, ws, (float *)dx);
    return hipGetLastError();
}

}  // namespace hos
