// k_c3.hip -- the third-order cumulant contraction on the gfx950 matrix cores.
//
// What is computed (Section 1, "Problem Statement": third-order moment of
// the mean-removed series, time average in place of the expectation):
//     C[a][b] = sum_i x_i x_{i+a} x_{i+b},   0 <= b <= a <= M,
// the fundamental region F of the six-fold lag symmetry; c3 on the whole
// hexagon is a relabelling of F (k_finish.hip).
//
// Formulation.  With r = a - 1, Y[r][i] = x_i x_{i+r+1} (the "product row")
// and the Hankel operand T[i][b] = x_{i+b}, C[r+1][b] = sum_i Y[r][i] T[i][b]
// is a dense (M x M) x n contraction.  Each wave owns up to 2 x 2 blocks of
// 32 x 32 outputs; the sample axis i is the MFMA k axis:
//   FP32 path   v_mfma_f32_32x32x2_f32, 8 per block per 16 samples;
//   split path  v_mfma_f32_32x32x16_{f16,bf16}, 3 per block per 16 samples
//               (Yhi*Thi + Yhi*Tlo + Ylo*Thi).
// Y is formed in registers from FP32 x (one multiply per element; the split
// rounds the exact FMA residual), T comes pre-split from the window tables.
// FP32 accumulators are flushed into FP64 registers after every chunk of
// KC = 512 samples; a workgroup's FP64 partial tile goes to the workspace
// and k_c3_reduce sums the partials of a tile in workgroup order.
//
// Staging.  Per chunk a workgroup copies three contiguous runs of 16-byte
// entries into LDS (prefetched into registers during the previous chunk's
// compute, double-buffered, one barrier per chunk):
//   s_xi  x_i, i in [i0, i0+KC)                       plain floats
//   s_xa  win4 entries [i0+r0, i0+r0+KC+TS)           rows' x_{i+r+1}
//   s_xb  win4 (FP32) or win8 hi|lo (split) entries [i0+b0, i0+b0+KC+TS)
// Entry o of a window table holds the 4 floats / 8 halves starting at
// sample o, so a lane's operand run x_{i+b .. i+b+7} is one (split) or two
// (FP32) aligned ds_read_b128 whatever its start sample, and consecutive
// lanes read consecutive entries (no bank conflicts).
#include "hos_internal.h"

namespace hos {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // promotable 16-byte unit

template <int PATH>
struct SplitOps;

// FP16 halves: hi = RNE16(y), lo = RNE16(fma(xi, xa, -hi)) (exact residual of
// the product, rounded once).
template <>
struct SplitOps<HOS_PATH_SPLIT_FP16> {
    typedef halfx8 vec;
    __device__ static inline void split(const float *xi, const float *xa, vec &h, vec &l)
    {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            _Float16 hh = (_Float16)(xi[j] * xa[j]);
            h[j] = hh;
            l[j] = (_Float16)__builtin_fmaf(xi[j], xa[j], -(float)hh);
        }
    }
    __device__ static inline vec from_bits(uint4 u) { return __builtin_bit_cast(vec, u); }
    __device__ static inline floatx16 mma(vec a, vec b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct SplitOps<HOS_PATH_SPLIT_BF16> {
    typedef bf16x8 vec;
    __device__ static inline void split(const float *xi, const float *xa, vec &h, vec &l)
    {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            __bf16 hh = (__bf16)(xi[j] * xa[j]);
            h[j] = hh;
            l[j] = (__bf16)__builtin_fmaf(xi[j], xa[j], -(float)hh);
        }
    }
    __device__ static inline vec from_bits(uint4 u) { return __builtin_bit_cast(vec, u); }
    __device__ static inline floatx16 mma(vec a, vec b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

__device__ inline void unpack8(float4 a, float4 b, float *v)
{
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// 32 k-groups of one staged chunk for one wave.  MASK bit (2*ra + rb) marks
// the active 32 x 32 blocks of the wave's 2 x 2 (WT = 2) or 1 x 1 window.
template <int PATH, int WT, int MASK>
__device__ inline void chunk_compute(const float4 *__restrict__ sxi,
                                     const float4 *__restrict__ sxa,
                                     const uint4 *__restrict__ sxb, int wlen,
                                     int rowbase, int colbase, int rl, int h,
                                     floatx16 (&acc)[WT][WT])
{
    constexpr bool SPLIT = PATH != HOS_PATH_FP32;
#pragma unroll 2
    for (int grp = 0; grp < KC / GROUP; ++grp) {
        const int ib = grp * GROUP + 8 * h;
        float xi[8];
        unpack8(sxi[ib >> 2], sxi[(ib >> 2) + 1], xi);
        if constexpr (SPLIT) {
            typedef SplitOps<PATH> Ops;
            typename Ops::vec yh[WT], yl[WT], th[WT], tl[WT];
#pragma unroll
            for (int ra = 0; ra < WT; ++ra) {
                if (!(MASK & (3 << (2 * ra))))
                    continue;
                const int o = ib + 32 * (rowbase + ra) + rl + 1;
                float xa[8];
                unpack8(sxa[o], sxa[o + 4], xa);
                Ops::split(xi, xa, yh[ra], yl[ra]);
            }
#pragma unroll
            for (int rb = 0; rb < WT; ++rb) {
                if (!(MASK & (5 << rb)))
                    continue;
                const int o = ib + 32 * (colbase + rb) + rl;
                th[rb] = Ops::from_bits(sxb[o]);
                tl[rb] = Ops::from_bits(sxb[wlen + o]);
            }
#pragma unroll
            for (int ra = 0; ra < WT; ++ra)
#pragma unroll
                for (int rb = 0; rb < WT; ++rb) {
                    if (!(MASK & (1 << (2 * ra + rb))))
                        continue;
                    acc[ra][rb] = Ops::mma(yh[ra], th[rb], acc[ra][rb]);
                    acc[ra][rb] = Ops::mma(yh[ra], tl[rb], acc[ra][rb]);
                    acc[ra][rb] = Ops::mma(yl[ra], th[rb], acc[ra][rb]);
                }
        } else {
            float y[WT][8], t[WT][8];
#pragma unroll
            for (int ra = 0; ra < WT; ++ra) {
                if (!(MASK & (3 << (2 * ra))))
                    continue;
                const int o = ib + 32 * (rowbase + ra) + rl + 1;
                float xa[8];
                unpack8(sxa[o], sxa[o + 4], xa);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    y[ra][j] = xi[j] * xa[j];
            }
#pragma unroll
            for (int rb = 0; rb < WT; ++rb) {
                if (!(MASK & (5 << rb)))
                    continue;
                const int o = ib + 32 * (colbase + rb) + rl;
                const float4 *sb = (const float4 *)sxb;
                unpack8(sb[o], sb[o + 4], t[rb]);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int ra = 0; ra < WT; ++ra)
#pragma unroll
                    for (int rb = 0; rb < WT; ++rb) {
                        if (!(MASK & (1 << (2 * ra + rb))))
                            continue;
                        acc[ra][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            y[ra][j], t[rb][j], acc[ra][rb], 0, 0, 0);
                    }
        }
    }
}

// Wave window inside a tile.  Off-diagonal tiles: wave w owns the 2x2 (WT=2)
// or 1x1 (WT=1) block window at (2*(w/2), 2*(w%2)) resp. (w/2, w%2).  In a
// diagonal WT=2 tile the 10 lower blocks are split 3/3/2/2 over the waves so
// that the tile costs 3 block-steps instead of 4.
__device__ inline void wave_window(int WT, bool diag, int wave, int tileR, int NBR,
                                   int &rowbase, int &colbase, int &mask)
{
    if (WT == 2) {
        if (!diag) {
            rowbase = 2 * (wave >> 1);
            colbase = 2 * (wave & 1);
            mask = 0xF;
        } else if (wave < 2) {
            rowbase = colbase = 2 * wave;
            mask = 0xD;           // (0,0) (1,0) (1,1)
        } else {
            rowbase = 2;
            colbase = wave - 2;
            mask = 0x5;           // (0,0) (1,0)
        }
    } else {
        rowbase = wave >> 1;
        colbase = wave & 1;
        mask = (diag && colbase > rowbase) ? 0 : 1;
    }
    // rows at or beyond NBR 32-blocks (r >= M rounded up) do not exist
    for (int ra = 0; ra < WT; ++ra)
        if (tileR * 2 * WT + rowbase + ra >= NBR)
            mask &= ~(3 << (2 * ra));
}

template <int PATH, int WT>
__device__ inline void dispatch_compute(int mask, const float4 *sxi, const float4 *sxa,
                                        const uint4 *sxb, int wlen, int rowbase, int colbase,
                                        int rl, int h, floatx16 (&acc)[WT][WT])
{
    if constexpr (WT == 2) {
        switch (mask) {
        case 0xF:
            chunk_compute<PATH, 2, 0xF>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
            break;
        case 0xD:
            chunk_compute<PATH, 2, 0xD>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
            break;
        case 0x5:
            chunk_compute<PATH, 2, 0x5>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
            break;
        case 0x3:
            chunk_compute<PATH, 2, 0x3>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
            break;
        case 0x1:
            chunk_compute<PATH, 2, 0x1>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
            break;
        default:
            break;  // 0: nothing to do
        }
    } else {
        if (mask & 1)
            chunk_compute<PATH, 1, 0x1>(sxi, sxa, sxb, wlen, rowbase, colbase, rl, h, acc);
    }
}

// One chunk's LDS operands (xi | xa | xb, contiguous 16-byte entries).
template <int PATH, int WT>
struct ChunkLds {
    static constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    static constexpr int TS = 64 * WT;
    static constexpr int WLEN = KC + TS;            // window entries per chunk
    static constexpr int NXI = KC / 4;              // float4 entries of x_i
    static constexpr int NXB = SPLIT ? 2 * WLEN : WLEN;
    static constexpr int TOTAL = NXI + WLEN + NXB;  // 16-byte entries
    static constexpr int NCH = TOTAL / 64;          // 1 KB wave-chunks
    static constexpr int NPW = (NCH + 3) / 4;       // wave-chunks per wave
    static_assert(NXI % 64 == 0 && WLEN % 64 == 0, "regions must be wave-chunk aligned");
    float4 xi[NXI];
    float4 xa[WLEN];
    uint4 xb[NXB];
};

// Global loads of one chunk into registers: wave-chunk j (64 consecutive
// 16-byte entries, one per lane) is handled by wave j % 4, so every branch
// below is wave-uniform and each load is a fully coalesced 1 KB read.
template <int PATH, int WT, int NPW>
__device__ __attribute__((always_inline)) inline void
load_chunk(u32x4 (&stg)[NPW], const float *__restrict__ xf,
           const uint4 *__restrict__ win4, const uint4 *__restrict__ win8h,
           const uint4 *__restrict__ win8l, const SkPos &p, int wave, int lane)
{
    typedef ChunkLds<PATH, WT> CL;
    const int64_t i0 = p.c * KC;
    const int64_t ra0 = i0 + (int64_t)p.R * CL::TS, rb0 = i0 + (int64_t)p.Cc * CL::TS;
    const u32x4 *xf4 = (const u32x4 *)xf;
    const u32x4 *w4 = (const u32x4 *)win4, *w8h = (const u32x4 *)win8h,
                *w8l = (const u32x4 *)win8l;
#pragma unroll
    for (int m = 0; m < CL::NPW; ++m) {
        const int j = wave + 4 * m;
        const int e = 64 * j;    // first entry of the wave-chunk
        const u32x4 *src;
        if (e < CL::NXI)
            src = xf4 + (i0 >> 2) + e;
        else if (e < CL::NXI + CL::WLEN)
            src = w4 + ra0 + (e - CL::NXI);
        else {
            const int e2 = e - CL::NXI - CL::WLEN;
            if (!CL::SPLIT)
                src = w4 + rb0 + e2;
            else if (e2 < CL::WLEN)
                src = w8h + rb0 + e2;
            else
                src = w8l + rb0 + (e2 - CL::WLEN);
        }
        if (j < CL::NCH)
            stg[m] = src[lane];
    }
}

template <int PATH, int WT, int NPW>
__device__ __attribute__((always_inline)) inline void
store_chunk(const u32x4 (&stg)[NPW], ChunkLds<PATH, WT> &L, int wave, int lane)
{
    typedef ChunkLds<PATH, WT> CL;
    u32x4 *base = (u32x4 *)&L;
#pragma unroll
    for (int m = 0; m < CL::NPW; ++m) {
        const int j = wave + 4 * m;
        if (j < CL::NCH)
            base[64 * j + lane] = stg[m];
    }
}

template <int PATH, int WT>
__device__ inline void flush_acc(floatx16 (&acc)[WT][WT], double (&acc64)[WT][WT][16])
{
#pragma unroll
    for (int ra = 0; ra < WT; ++ra)
#pragma unroll
        for (int rb = 0; rb < WT; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc64[ra][rb][v] += (double)acc[ra][rb][v];
                acc[ra][rb][v] = 0.0f;
            }
}

template <int PATH, int WT>
__global__ void __launch_bounds__(256, 1)
k_c3_contract(const float *__restrict__ xf, const uint4 *__restrict__ win4,
              const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l,
              double *__restrict__ part, SkGeom g, int64_t smax, int NBR)
{
    typedef ChunkLds<PATH, WT> CL;
    constexpr int NB = 2 * WT;                    // 32-blocks per tile side
    constexpr int64_t TILE = (int64_t)CL::TS * CL::TS;

    __shared__ CL buf[2];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, rl = lane & 31, h = lane >> 5;
    const int64_t w = blockIdx.x;
    const int64_t S0 = sk_wg_start(g, w), S1 = sk_wg_start(g, w + 1);

    SkPos q;
    if (!sk_first_chunk(g, S0, q) || sk_chunk_start(g, q.R, q.Cc, q.c) >= S1)
        return;
    const int64_t tfirst = sk_tile_index(q.R, q.Cc);

    floatx16 acc[WT][WT];
    double acc64[WT][WT][16];
#pragma unroll
    for (int ra = 0; ra < WT; ++ra)
#pragma unroll
        for (int rb = 0; rb < WT; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[ra][rb][v] = 0.0f;
                acc64[ra][rb][v] = 0.0;
            }

    int rowbase, colbase, mask;
    wave_window(WT, q.Cc == q.R, wave, q.R, NBR, rowbase, colbase, mask);
    mask = __builtin_amdgcn_readfirstlane(mask);
    rowbase = __builtin_amdgcn_readfirstlane(rowbase);
    colbase = __builtin_amdgcn_readfirstlane(colbase);

    u32x4 stg[CL::NPW];
    load_chunk<PATH, WT, CL::NPW>(stg, xf, win4, win8h, win8l, q, wave, lane);
    store_chunk<PATH, WT, CL::NPW>(stg, buf[0], wave, lane);
    __syncthreads();

    // Each step prefetches the next chunk into registers, computes on the
    // current LDS buffer, flushes FP32 -> FP64, writes the partial tile at a
    // segment end, then stores the prefetched chunk into the other buffer.
    // One barrier per chunk: a buffer is rewritten only after every wave has
    // passed the barrier that follows its last use.
    int cur = 0;
    for (;;) {
        SkPos nq = q;
        const bool has_next = sk_next(g, nq) && sk_chunk_start(g, nq.R, nq.Cc, nq.c) < S1;
        if (has_next)
            load_chunk<PATH, WT, CL::NPW>(stg, xf, win4, win8h, win8l, nq, wave, lane);

        dispatch_compute<PATH, WT>(mask, buf[cur].xi, buf[cur].xa, buf[cur].xb, CL::WLEN,
                                   rowbase, colbase, rl, h, acc);
        flush_acc<PATH, WT>(acc, acc64);

        const bool seg_end = !has_next || nq.R != q.R || nq.Cc != q.Cc;
        if (seg_end) {
            const int64_t t = sk_tile_index(q.R, q.Cc);
            double *dst = part + (w * smax + (t - tfirst)) * TILE;
#pragma unroll
            for (int ra = 0; ra < WT; ++ra)
#pragma unroll
                for (int rb = 0; rb < WT; ++rb) {
                    if (mask & (1 << (2 * ra + rb))) {
                        const int blk = (rowbase + ra) * NB + (colbase + rb);
#pragma unroll
                        for (int v = 0; v < 16; ++v)
                            dst[(blk * 16 + v) * 64 + lane] = acc64[ra][rb][v];
                    }
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        acc64[ra][rb][v] = 0.0;
                }
        }
        if (!has_next)
            break;
        cur ^= 1;
        store_chunk<PATH, WT, CL::NPW>(stg, buf[cur], wave, lane);
        __syncthreads();
        if (seg_end) {
            wave_window(WT, nq.Cc == nq.R, wave, nq.R, NBR, rowbase, colbase, mask);
            mask = __builtin_amdgcn_readfirstlane(mask);
            rowbase = __builtin_amdgcn_readfirstlane(rowbase);
            colbase = __builtin_amdgcn_readfirstlane(colbase);
        }
        q = nq;
    }
}

// Sum the FP64 partial tiles of every workgroup that touched the tile, in
// workgroup order, and scatter the 32 x 32 block to Cfull[a][b] (a = r + 1).
// One workgroup per (tile, 32-block).
template <int WT>
__global__ void __launch_bounds__(256)
k_c3_reduce(const double *__restrict__ part, SkGeom g, int64_t smax, int NBR, int M,
            double *__restrict__ cfull)
{
    constexpr int NB = 2 * WT;
    constexpr int64_t TILE = (int64_t)(64 * WT) * (64 * WT);
    const int64_t t = blockIdx.x / (NB * NB);
    const int blk = blockIdx.x % (NB * NB);
    int R = 0;
    while (sk_tile_index(R + 1, 0) <= t)
        ++R;
    const int Cc = (int)(t - sk_tile_index(R, 0));
    const int bR = blk / NB, bC = blk % NB;
    const int Rg = R * NB + bR, Bg = Cc * NB + bC;
    if (Rg >= NBR || Bg > Rg)
        return;
    const int64_t w_lo = sk_owner(g, sk_chunk_start(g, R, Cc, 0));
    const int64_t w_hi = sk_owner(g, sk_chunk_start(g, R, Cc, g.C - 1));
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t w = w_lo; w <= w_hi; ++w) {
        SkPos p;
        sk_first_chunk(g, sk_wg_start(g, w), p);
        const int64_t slot = w * smax + (t - sk_tile_index(p.R, p.Cc));
        const double *src = part + slot * TILE + (int64_t)blk * 1024;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            sum[k] += src[threadIdx.x + 256 * k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int v = e >> 6, lane = e & 63;
        // 32x32 MFMA accumulator layout: column = lane % 32,
        // row = 8 (v / 4) + 4 (lane / 32) + v % 4
        const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = lane & 31;
        const int r = Rg * 32 + row, b = Bg * 32 + col;
        if (r < M && (Bg < Rg || col <= row + 1))
            cfull[(int64_t)(r + 1) * (M + 1) + b] = sum[k];
    }
}

// Leftover diagonal sums C[a][a] = sum_i x_i x_{i+a}^2 for a = 0 and
// a = 32k <= M, in FP64 from the FP32 operand series (fixed-order partials).
__global__ void __launch_bounds__(256)
k_diag_dot(const float *__restrict__ xf, int64_t n, int nblocks, double *__restrict__ dpart)
{
    __shared__ double red[256];
    const int left = blockIdx.x / nblocks, blk = blockIdx.x % nblocks;
    const int64_t a = 32 * (int64_t)left;
    double s = 0.0;
    for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < n; i += (int64_t)nblocks * 256) {
        const double u = xf[i + a];
        s += (double)xf[i] * u * u;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        if (threadIdx.x < wdt)
            red[threadIdx.x] += red[threadIdx.x + wdt];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        dpart[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(64)
k_diag_final(const double *__restrict__ dpart, int nleft, int nblocks, int M,
             double *__restrict__ cfull)
{
    const int left = blockIdx.x * 64 + threadIdx.x;
    if (left >= nleft)
        return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b)
        s += dpart[left * nblocks + b];
    const int64_t a = 32 * (int64_t)left;
    cfull[a * (M + 1) + a] = s;
}

template <int PATH, int WT>
void launch_contract_t(const C3Plan &p, char *ws, hipStream_t s)
{
    k_c3_contract<PATH, WT><<<p.sk.G, WG_THREADS, 0, s>>>(
        (const float *)(ws + p.off_xf), (const uint4 *)(ws + p.off_win4),
        (const uint4 *)(ws + p.off_win8h), (const uint4 *)(ws + p.off_win8l),
        (double *)(ws + p.off_part), p.sk, p.smax, p.NBR);
}

}  // namespace

hipError_t launch_c3_contract(const C3Plan &p, char *ws, hipStream_t s)
{
    if (p.M > 0) {
        if (p.WT == 2) {
            if (p.path == HOS_PATH_FP32)
                launch_contract_t<HOS_PATH_FP32, 2>(p, ws, s);
            else if (p.path == HOS_PATH_SPLIT_FP16)
                launch_contract_t<HOS_PATH_SPLIT_FP16, 2>(p, ws, s);
            else
                launch_contract_t<HOS_PATH_SPLIT_BF16, 2>(p, ws, s);
        } else {
            if (p.path == HOS_PATH_FP32)
                launch_contract_t<HOS_PATH_FP32, 1>(p, ws, s);
            else if (p.path == HOS_PATH_SPLIT_FP16)
                launch_contract_t<HOS_PATH_SPLIT_FP16, 1>(p, ws, s);
            else
                launch_contract_t<HOS_PATH_SPLIT_BF16, 1>(p, ws, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_diag_dot(const C3Plan &p, char *ws, hipStream_t s)
{
    k_diag_dot<<<p.nleft * p.dot_blocks, 256, 0, s>>>((const float *)(ws + p.off_xf), p.n,
                                                     p.dot_blocks,
                                                     (double *)(ws + p.off_dpart));
    return hipGetLastError();
}

hipError_t launch_c3_reduce(const C3Plan &p, char *ws, hipStream_t s)
{
    double *cfull = (double *)(ws + p.off_cfull);
    if (p.M > 0) {
        const int64_t ntiles = (int64_t)p.sk.TR * (p.sk.TR + 1) / 2;
        const int NB = 2 * p.WT;
        if (p.WT == 2)
            k_c3_reduce<2><<<ntiles * NB * NB, 256, 0, s>>>((const double *)(ws + p.off_part),
                                                          p.sk, p.smax, p.NBR, p.M, cfull);
        else
            k_c3_reduce<1><<<ntiles * NB * NB, 256, 0, s>>>((const double *)(ws + p.off_part),
                                                          p.sk, p.smax, p.NBR, p.M, cfull);
    }
    k_diag_final<<<(p.nleft + 63) / 64, 64, 0, s>>>((const double *)(ws + p.off_dpart),
                                                   p.nleft, p.dot_blocks, p.M, cfull);
    return hipGetLastError();
}

}  // namespace hos
