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
// FP32 accumulators are flushed into FP64 registers after every staged chunk
// (KC = 512 samples; 2 KC on the split paths' 4-block tiles); a workgroup's
// FP64 partial tile goes to the workspace and k_c3_reduce sums the partials
// of a tile in workgroup order.
//
// Staging.  Per chunk a workgroup copies three contiguous runs of 16-byte
// entries into LDS (prefetched during the previous chunk's compute -- through
// registers, or on the split paths straight into LDS -- double-buffered, one
// barrier per chunk):
//   s_xi  x_i, i in [i0, i0+L)                        plain floats
//   s_xa  win4 entries [i0+r0, i0+r0+L+TS)            rows' x_{i+r+1}
//   s_xb  win4 (FP32) or win8 hi|lo (split) entries [i0+b0, i0+b0+L+TS)
// with L the chunk length; a chunk of 2 KC is computed as two KC sub-chunks
// whose runs start KC entries apart.
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

// FP16 halves of the product y = xi * xa: hi = RNE16(fl32(y)) by one
// packed conversion per two elements, and lo = RNE16(y - hi) by one fused
// multiply-add per element straight from the exact product
// (v_fma_mix{lo,hi}_f16 round a full-precision fma to FP16 and write one
// half of a packed register); |y - hi - lo| <= 2^-22 |y|.  The mixed FMA
// issues at about a third of the FP32 FMA rate on this chip, so hi comes
// from the FP32 product and the conversion instead (2 multiplies + 1
// conversion in place of 2 mixed FMAs per two elements).
template <>
struct SplitOps<HOS_PATH_SPLIT_FP16> {
    typedef halfx8 vec;
    __device__ static inline void split(const float *xi, const float *xa, vec &h, vec &l)
    {
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t hv, lv;
            const float y0 = xi[2 * p] * xa[2 * p], y1 = xi[2 * p + 1] * xa[2 * p + 1];
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hv) : "v"(y0), "v"(y1));
            asm("v_fma_mixlo_f16 %0, %1, %2, -%3 op_sel_hi:[0,0,1]"
                : "=v"(lv) : "v"(xi[2 * p]), "v"(xa[2 * p]), "v"(hv));
            asm("v_fma_mixhi_f16 %0, %1, %2, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
                : "+v"(lv) : "v"(xi[2 * p + 1]), "v"(xa[2 * p + 1]), "v"(hv));
            hw[p] = hv;
            lw[p] = lv;
        }
        h = __builtin_bit_cast(vec, hw);
        l = __builtin_bit_cast(vec, lw);
    }
    __device__ static inline vec from_bits(uint4 u) { return __builtin_bit_cast(vec, u); }
    __device__ static inline floatx16 mma(vec a, vec b, floatx16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// BF16 halves: hi = RNE_bf16(y), lo = RNE_bf16(fma(xi, xa, -hi)).
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

// The FP64 accumulators are touched once per flush, so they are kept in the
// accumulation register file (AGPRs): the empty asm pins each value to an
// AGPR after its update, leaving the VGPRs to the operand pipeline.
__device__ __attribute__((always_inline)) inline void pin_agpr(double &v)
{
    asm volatile("" : "+a"(v));
}

// sgn = -1 undoes the negated product rows of an odd chunk (see below).
// The first NB of the NA accumulator blocks are flushed.
template <int NB, bool PIN, int NA = NB>
__device__ inline void flush_acc(floatx16 (&acc)[NA], double (&acc64)[NA][16], float sgn)
{
    static_assert(NB <= NA, "flushing more blocks than the arrays hold");
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc64[cb][v] += (double)(sgn * acc[cb][v]);
            if (PIN)
                pin_agpr(acc64[cb][v]);
            acc[cb][v] = 0.0f;
        }
}

// FP32 partial sums move into FP64 every FlushPeriod::GROUPS k-groups.  The
// matrix-core FP32 accumulation error grows linearly with the length of the
// chain (measured: the bias of each add is relative to the running sum), and
// a cumulant that is pure sampling noise (Gaussian input) sits far below the
// size of its terms, so the chain length sets the relative error there.
//
// The error also has a direction: measured on gfx950, a matrix-core op that
// sums products of mixed sign is biased toward -infinity (about -0.6 to
// -2.7 ulp of its result for FP16 inputs, -0.05 ulp for FP32), whatever
// the sign of the result.  Summed over every chunk and then over every lag
// by the DFT, that bias would add up coherently.  Odd chunks therefore run
// on negated x_i (so every product row, and the chunk's sum, changes sign;
// the negation is exact) and are flushed with sgn = -1: their bias points
// the other way and the two halves cancel.
template <int PATH>
struct FlushPeriod {
    static constexpr int GROUPS = PATH == HOS_PATH_FP32 ? 4 : KC / GROUP;
};

// Row-side operands of one 16-sample k-group as read from LDS: x_i and the
// wave's run x_{i+r+1} (8 samples per lane).
struct RowRaw {
    float4 xi0, xi1, xa0, xa1;
};

__device__ __attribute__((always_inline)) inline void
fetch_rows(RowRaw &r, const float4 *__restrict__ sxi, const float4 *__restrict__ sxa, int grp,
           int rw, int rl, int h)
{
    const int ib = grp * GROUP + 8 * h;
    const int o = ib + 32 * rw + rl + 1;
    r.xi0 = sxi[ib >> 2];
    r.xi1 = sxi[(ib >> 2) + 1];
    r.xa0 = sxa[o];
    r.xa1 = sxa[o + 4];
}

// Hankel windows.  Column block cb of group g needs T[i][b] = x_{i+b} for
// the lane's 8 samples i = i0 + 16g + 8h + j and b = b0 + 32cb + rl, i.e. the
// window table entry at o = 16(g + 2cb) + 8h + rl.  Writing V[u] for the
// entry at 16u + 8h + rl, group g uses V[g], V[g+2], .., V[g+2(NCOL-1)]:
// group g+2 reuses all but one of group g's windows, so each group loads a
// single new window instead of NCOL.  A window is two 16-byte entries --
// split: T hi, T lo; FP32: T[0..3], T[4..7].
struct Win {
    uint4 a, b;
};

template <int PATH>
__device__ __attribute__((always_inline)) inline void
fetch_win(Win &v, const uint4 *__restrict__ sxb, int wlen, int u, int rl, int h)
{
    const int o = 16 * u + 8 * h + rl;
    v.a = sxb[o];
    v.b = PATH == HOS_PATH_FP32 ? sxb[o + 4] : sxb[wlen + o];
}

template <int PATH>
struct Yrow {
    typename SplitOps<PATH>::vec yh, yl;
};

template <int PATH>
__device__ __attribute__((always_inline)) inline void split_rows(Yrow<PATH> &y, const RowRaw &r)
{
    float xi[8], xa[8];
    unpack8(r.xi0, r.xi1, xi);
    unpack8(r.xa0, r.xa1, xa);
    SplitOps<PATH>::split(xi, xa, y.yh, y.yl);
}

// One staged chunk (KC samples = 32 k-groups, fully unrolled so that the
// window ring and the pipeline stages have fixed registers) for one wave:
// its 32-row strip rw against the first NCOL column blocks.  At step g the
// wave issues the LDS reads of window V[g + 2 NCOL] and of the rows of group
// g+2, splits the product row of group g+1, and runs group g's matrix-core
// ops.  The fences keep each step's LDS reads ahead of its matrix-core ops
// (the compiler would otherwise sink them next to their consumers and expose
// the LDS latency); only VALU ops may cross them, so the split interleaves
// with the matrix-core ops.  The FP32 path has the same structure with one
// multiply per product and 8 matrix-core steps per block per group.
template <int PATH, int NB, int NCOL, int NA = NB, int NG = KC / GROUP>
__device__ __attribute__((always_inline)) inline void chunk_compute(const float4 *__restrict__ sxi,
                                     const float4 *__restrict__ sxa,
                                     const uint4 *__restrict__ sxb, int wlen, int rw, int rl,
                                     int h, floatx16 (&acc)[NA], double (&acc64)[NA][16])
{
    static_assert(NCOL <= NB && NB <= NA, "column blocks beyond the accumulator arrays");
    constexpr int UMAX = NG - 1 + 2 * (NCOL - 1);   // last window used
    constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    if constexpr (SPLIT) {
        typedef SplitOps<PATH> Ops;
        Win V[UMAX + 1];
        RowRaw raw[NG];
#pragma unroll
        for (int u = 0; u < 2 * NCOL && u <= UMAX; ++u)
            fetch_win<PATH>(V[u], sxb, wlen, u, rl, h);
        fetch_rows(raw[0], sxi, sxa, 0, rw, rl, h);
        fetch_rows(raw[1], sxi, sxa, 1, rw, rl, h);
        Yrow<PATH> Y[NG];
        split_rows<PATH>(Y[0], raw[0]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g + 2 * NCOL <= UMAX)
                fetch_win<PATH>(V[g + 2 * NCOL], sxb, wlen, g + 2 * NCOL, rl, h);
            if (g + 2 < NG)
                fetch_rows(raw[g + 2], sxi, sxa, g + 2, rw, rl, h);
            if (g + 1 < NG)
                split_rows<PATH>(Y[g + 1], raw[g + 1]);
            __builtin_amdgcn_sched_barrier(0x0002);
            // term-major: consecutive matrix-core ops write different accumulators
#pragma unroll
            for (int term = 0; term < 3; ++term)
#pragma unroll
                for (int cb = 0; cb < NCOL; ++cb) {
                    const Win &w = V[g + 2 * cb];
                    acc[cb] = Ops::mma(term == 2 ? Y[g].yl : Y[g].yh,
                                       Ops::from_bits(term == 1 ? w.b : w.a), acc[cb]);
                }
            __builtin_amdgcn_sched_barrier(0x0002);
        }
    } else {
        static_assert(SPLIT, "the FP32 path uses chunk_compute_fp32");
    }
}

// FP32 path: each wave owns a 2 x 2 window of 32 x 32 blocks (rows
// rowbase, rowbase+1; columns colbase, colbase+1 of the tile), MASK bit
// (2 ra + rb) marking the active ones.  8 matrix-core steps per block per
// 16-sample group; the operands of group g+1 are read while group g runs.
template <int MASK>
__device__ __attribute__((always_inline)) inline void chunk_compute_fp32(const float4 *__restrict__ sxi,
                                          const float4 *__restrict__ sxa,
                                          const uint4 *__restrict__ sxb, int rowbase,
                                          int colbase, int rl, int h, floatx16 (&acc)[4],
                                          double (&acc64)[4][16], float sgn)
{
    constexpr int NG = KC / GROUP;
    constexpr int FG = FlushPeriod<HOS_PATH_FP32>::GROUPS;
    constexpr bool R0 = (MASK & 3) != 0, R1 = (MASK & 12) != 0;
    constexpr bool C0 = (MASK & 5) != 0, C1 = (MASK & 10) != 0;
    auto fetch = [&](int g, RowRaw (&rr)[2], Win (&tt)[2]) __attribute__((always_inline)) {
        fetch_rows(rr[0], sxi, sxa, g, rowbase, rl, h);
        if (R1) {
            const int ib = g * GROUP + 8 * h;
            const int o = ib + 32 * (rowbase + 1) + rl + 1;
            rr[1].xa0 = sxa[o];
            rr[1].xa1 = sxa[o + 4];
        }
        if (C0)
            fetch_win<HOS_PATH_FP32>(tt[0], sxb, 0, g + 2 * colbase, rl, h);
        if (C1)
            fetch_win<HOS_PATH_FP32>(tt[1], sxb, 0, g + 2 * colbase + 2, rl, h);
    };
    RowRaw r[2], rn[2];
    Win t[2], tn[2];
    fetch(0, r, t);
#pragma unroll 1
    for (int g = 0; g < NG; ++g) {
        fetch((g + 1) & (NG - 1), rn, tn);   // wraps to a valid, unused group
        float xi[8], y[2][8], tv[2][8];
        unpack8(r[0].xi0, r[0].xi1, xi);
#pragma unroll
        for (int ra = 0; ra < 2; ++ra) {
            float xa[8];
            unpack8(r[ra].xa0, r[ra].xa1, xa);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                y[ra][j] = xi[j] * xa[j];
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
            unpack8(__builtin_bit_cast(float4, t[rb].a), __builtin_bit_cast(float4, t[rb].b),
                    tv[rb]);
        __builtin_amdgcn_sched_barrier(0x0002);
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int ra = 0; ra < 2; ++ra)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
                    if (MASK & (1 << (2 * ra + rb)))
                        acc[2 * ra + rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            y[ra][j], tv[rb][j], acc[2 * ra + rb], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0x0002);
        r[0] = rn[0];
        r[1] = rn[1];
        t[0] = tn[0];
        t[1] = tn[1];
        if ((g + 1) % FG == 0)
            flush_acc<4, false>(acc, acc64, sgn);
    }
}

// FP32 wave window inside a 128 x 128 tile.  Off the diagonal wave w owns the
// 2 x 2 blocks at (2 (w/2), 2 (w%2)); on a diagonal tile the 10 blocks on or
// below the diagonal are split 3/3/2/2 so the tile costs 3 block-steps.
__device__ inline void fp32_window(bool diag, int wave, int tileR, int NBR, int &rowbase,
                                   int &colbase, int &mask)
{
    if (!diag) {
        rowbase = 2 * (wave >> 1);
        colbase = 2 * (wave & 1);
        mask = 0xF;
    } else if (wave < 2) {
        rowbase = colbase = 2 * wave;
        mask = 0xD;   // (0,0) (1,0) (1,1)
    } else {
        rowbase = 2;
        colbase = wave - 2;
        mask = 0x5;   // (0,0) (1,0)
    }
    for (int ra = 0; ra < 2; ++ra)
        if (tileR * 4 + rowbase + ra >= NBR)
            mask &= ~(3 << (2 * ra));
}

__device__ __attribute__((always_inline)) inline void dispatch_fp32(int mask, const float4 *sxi, const float4 *sxa,
                                     const uint4 *sxb, int rowbase, int colbase, int rl, int h,
                                     floatx16 (&acc)[4], double (&acc64)[4][16], float sgn)
{
    switch (mask) {
    case 0xF: chunk_compute_fp32<0xF>(sxi, sxa, sxb, rowbase, colbase, rl, h, acc, acc64, sgn); break;
    case 0xD: chunk_compute_fp32<0xD>(sxi, sxa, sxb, rowbase, colbase, rl, h, acc, acc64, sgn); break;
    case 0x5: chunk_compute_fp32<0x5>(sxi, sxa, sxb, rowbase, colbase, rl, h, acc, acc64, sgn); break;
    case 0x3: chunk_compute_fp32<0x3>(sxi, sxa, sxb, rowbase, colbase, rl, h, acc, acc64, sgn); break;
    case 0x1: chunk_compute_fp32<0x1>(sxi, sxa, sxb, rowbase, colbase, rl, h, acc, acc64, sgn); break;
    default: break;
    }
}

// Active column blocks of wave rw's strip in a tile: all NB off the
// diagonal, rw + 1 on a diagonal tile (blocks above it are outside F), none
// for strips at or beyond the last 32-row block (rows r >= M).
__device__ inline int wave_cols(int NB, bool diag, int rw, int tileR, int NBR)
{
    if (tileR * NB + rw >= NBR)
        return 0;
    return diag ? rw + 1 : NB;
}

// NB: column blocks of the tile; the accumulator arrays hold NA >= NB blocks;
// NG: 16-sample groups (a KC-sample run by default).
template <int PATH, int NB, int NA = NB, int NG = KC / GROUP>
__device__ __attribute__((always_inline)) inline void dispatch_compute(int ncol, const float4 *sxi, const float4 *sxa,
                                        const uint4 *sxb, int wlen, int rw, int rl, int h,
                                        floatx16 (&acc)[NA], double (&acc64)[NA][16])
{
    switch (ncol) {
    case 1:
        chunk_compute<PATH, NB, 1, NA, NG>(sxi, sxa, sxb, wlen, rw, rl, h, acc, acc64);
        break;
    case 2:
        chunk_compute<PATH, NB, 2, NA, NG>(sxi, sxa, sxb, wlen, rw, rl, h, acc, acc64);
        break;
    case 3:
        if constexpr (NB >= 3)
            chunk_compute<PATH, NB, 3, NA, NG>(sxi, sxa, sxb, wlen, rw, rl, h, acc, acc64);
        break;
    case 4:
        if constexpr (NB >= 4)
            chunk_compute<PATH, NB, 4, NA, NG>(sxi, sxa, sxb, wlen, rw, rl, h, acc, acc64);
        break;
    default:
        break;  // 0: this strip has no output in the tile
    }
}

// One chunk's LDS operands (xi | xa | xb, contiguous 16-byte entries) for
// a tile of NB x NB blocks, staged by a workgroup of NWG waves.
template <int PATH, int NB, int KCX = KC, int NWG = NB>
struct ChunkLds {
    static constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    static constexpr int NW = NWG;                  // waves per workgroup
    static constexpr int TS = 32 * NB;
    static constexpr int WLEN = KCX + TS;           // window entries per chunk
    static constexpr int NXI = KCX / 4;             // float4 entries of x_i
    static constexpr int NXB = SPLIT ? 2 * WLEN : WLEN;
    static constexpr int TOTAL = NXI + WLEN + NXB;  // 16-byte entries
    static constexpr int NCH = TOTAL / 64;          // 1 KB wave-chunks
    static constexpr int NPW = (NCH + NW - 1) / NW; // wave-chunks per wave
    static_assert(NXI % 64 == 0 && WLEN % 64 == 0, "regions must be wave-chunk aligned");
    float4 xi[NXI];
    float4 xa[WLEN];
    uint4 xb[NXB];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // promotable 16-byte unit

// Global loads of one chunk into registers: wave-chunk j (64 consecutive
// 16-byte entries, one per lane) is handled by wave j % NW, so every branch
// below is wave-uniform and each load is a fully coalesced 1 KB read.
template <int PATH, int NB, int NPW>
__device__ __attribute__((always_inline)) inline void
load_chunk(u32x4 (&stg)[NPW], const float *__restrict__ xf, const uint4 *__restrict__ win4,
           const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l, const SkPos &p,
           int wave, int lane, int64_t coff)
{
    typedef ChunkLds<PATH, NB> CL;
    const int64_t i0 = p.c * KC;
    const int64_t ra0 = i0 + (int64_t)p.R * CL::TS, rb0 = i0 + (int64_t)p.Cc * CL::TS + coff;
    const u32x4 *xf4 = (const u32x4 *)xf;
    const u32x4 *w4 = (const u32x4 *)win4, *w8h = (const u32x4 *)win8h,
                *w8l = (const u32x4 *)win8l;
#pragma unroll
    for (int m = 0; m < NPW; ++m) {
        const int j = wave + CL::NW * m;
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

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// Split paths of the single-series kernel: the window regions go straight
// from global memory into the LDS buffer (gfx950's 16-byte global_load_lds:
// lane l writes entry l of the wave-chunk, the same layout store_chunk
// writes), which frees the staging registers; only the x_i run, whose sign
// depends on the chunk's parity, passes through registers.  The loads land in
// the buffer the workgroup is not computing on; store_xi waits for them
// before the barrier that hands the buffer over.
template <int N>
struct XiRegsN {
    u32x4 r[N];
};
template <class CL>
using XiRegs = XiRegsN<(CL::NXI / 64 + CL::NW - 1) / CL::NW>;

template <class CL>
__device__ __attribute__((always_inline)) inline void
load_chunk_dma(XiRegs<CL> &xr, const float *__restrict__ xf, const uint4 *__restrict__ win4,
               const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l, const SkPos &p,
               CL &L, int wave, int lane, int64_t coff)
{
    constexpr int KCX = CL::NXI * 4;
    const int64_t i0 = p.c * KCX;
    const int64_t ra0 = i0 + (int64_t)p.R * CL::TS, rb0 = i0 + (int64_t)p.Cc * CL::TS + coff;
    const u32x4 *xf4 = (const u32x4 *)xf;
    const u32x4 *w4 = (const u32x4 *)win4, *w8h = (const u32x4 *)win8h,
                *w8l = (const u32x4 *)win8l;
    u32x4 *base = (u32x4 *)&L;
#pragma unroll
    for (int m = 0; m < CL::NPW; ++m) {
        const int j = wave + CL::NW * m;
        const int e = 64 * j;
        if (j >= CL::NCH)
            continue;
        if (e < CL::NXI) {
            if (m < (int)(sizeof(xr.r) / sizeof(xr.r[0])))
                xr.r[m] = xf4[(i0 >> 2) + e + lane];
            continue;
        }
        const u32x4 *src;
        if (e < CL::NXI + CL::WLEN)
            src = w4 + ra0 + (e - CL::NXI);
        else {
            const int e2 = e - CL::NXI - CL::WLEN;
            src = e2 < CL::WLEN ? w8h + rb0 + e2 : w8l + rb0 + (e2 - CL::WLEN);
        }
        __builtin_amdgcn_global_load_lds((glb_void_t *)(src + lane), (lds_void_t *)(base + e), 16,
                                         0, 0);
    }
}

template <class CL>
__device__ __attribute__((always_inline)) inline void
store_xi(const XiRegs<CL> &xr, CL &L, int wave, int lane, bool neg)
{
    u32x4 *base = (u32x4 *)&L;
#pragma unroll
    for (int m = 0; m < (int)(sizeof(xr.r) / sizeof(xr.r[0])); ++m) {
        const int j = wave + CL::NW * m;
        if (64 * j < CL::NXI)
            base[64 * j + lane] = xr.r[m] ^ (neg ? 0x80000000u : 0u);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// neg: store the x_i run with its sign flipped (odd chunks).
template <int PATH, int NB, int NPW>
__device__ __attribute__((always_inline)) inline void
store_chunk(const u32x4 (&stg)[NPW], ChunkLds<PATH, NB> &L, int wave, int lane, bool neg)
{
    typedef ChunkLds<PATH, NB> CL;
    u32x4 *base = (u32x4 *)&L;
    const unsigned flip = neg ? 0x80000000u : 0u;
#pragma unroll
    for (int m = 0; m < NPW; ++m) {
        const int j = wave + CL::NW * m;
        if (j < CL::NCH)
            base[64 * j + lane] = 64 * j < CL::NXI ? (stg[m] ^ flip) : stg[m];
    }
}

// The persistent contraction kernel: NB waves per workgroup, wave rw owning
// the 32-row strip rw of every tile it visits.  coff shifts the Hankel
// columns: 0 for the fundamental region (column b = sample offset b), M + 1
// for the square's corners (column c = sample offset M + 1 + c, the same
// lower-triangular tile set since a corner sum needs c <= r).
template <int PATH, int NB>
__global__ void __launch_bounds__(64 * NB, 1)
k_c3_contract(const float *__restrict__ xf, const uint4 *__restrict__ win4,
              const uint4 *__restrict__ win8h, const uint4 *__restrict__ win8l,
              double *__restrict__ part, SkGeom g, int64_t smax, int NBR, int64_t coff)
{
    constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    // samples staged per barrier: split paths with 4-block tiles stage two
    // KC-sample sub-chunks at once (116 KB of LDS), which halves the
    // barriers, prologues and FP64 flushes per sample
    constexpr int KCX = c3_stage_len(PATH, NB);
    typedef ChunkLds<PATH, NB, KCX> CL;
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

    floatx16 acc[NB];
    double acc64[NB][16];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc[cb][v] = 0.0f;
            acc64[cb][v] = 0.0;
            if (PATH != HOS_PATH_FP32)
                pin_agpr(acc64[cb][v]);
        }

    // split paths: wave = row strip with ncol column blocks; FP32: 2 x 2 window
    int ncol = 0, rowbase = 0, colbase = 0, mask = 0;
    auto set_layout = [&](const SkPos &p) {
        if constexpr (PATH == HOS_PATH_FP32) {
            fp32_window(p.Cc == p.R, wave, p.R, NBR, rowbase, colbase, mask);
            mask = __builtin_amdgcn_readfirstlane(mask);
            rowbase = __builtin_amdgcn_readfirstlane(rowbase);
            colbase = __builtin_amdgcn_readfirstlane(colbase);
        } else {
            ncol = __builtin_amdgcn_readfirstlane(wave_cols(NB, p.Cc == p.R, wave, p.R, NBR));
        }
    };
    set_layout(q);

    u32x4 stg[CL::NPW];
    XiRegs<CL> xr;
    if constexpr (!SPLIT) {
        load_chunk<PATH, NB, CL::NPW>(stg, xf, win4, win8h, win8l, q, wave, lane, coff);
        store_chunk<PATH, NB, CL::NPW>(stg, buf[0], wave, lane, q.c & 1);
    } else {
        load_chunk_dma<CL>(xr, xf, win4, win8h, win8l, q, buf[0], wave, lane, coff);
        store_xi<CL>(xr, buf[0], wave, lane, q.c & 1);
    }
    __syncthreads();

    // Each step prefetches the next chunk (into registers, or for the split
    // paths straight into the other LDS buffer), computes on the current
    // buffer, flushes FP32 -> FP64, writes the partial tile at a segment end,
    // then stores the prefetched chunk (the split paths: its x_i run).
    // One barrier per chunk: a buffer is rewritten only after every wave has
    // passed the barrier that follows its last use.
    int cur = 0;
    for (;;) {
        SkPos nq = q;
        const bool has_next = sk_next(g, nq) && sk_chunk_start(g, nq.R, nq.Cc, nq.c) < S1;
        if (has_next) {
            if constexpr (!SPLIT)
                load_chunk<PATH, NB, CL::NPW>(stg, xf, win4, win8h, win8l, nq, wave, lane, coff);
            else
                load_chunk_dma<CL>(xr, xf, win4, win8h, win8l, nq, buf[cur ^ 1],
                                              wave, lane, coff);
        }

        const float sgn = (q.c & 1) ? -1.0f : 1.0f;
        if constexpr (PATH == HOS_PATH_FP32) {
            static_assert(NB == 4, "the FP32 wave layout assumes 4 x 4-block tiles");
            dispatch_fp32(mask, buf[cur].xi, buf[cur].xa, buf[cur].xb, rowbase, colbase, rl, h,
                          acc, acc64, sgn);
        } else {
            dispatch_compute<PATH, NB>(ncol, buf[cur].xi, buf[cur].xa, buf[cur].xb, CL::WLEN,
                                       wave, rl, h, acc, acc64);
            if constexpr (KCX == 2 * KC)   // the second sub-chunk: every run shifted by KC
                dispatch_compute<PATH, NB>(ncol, buf[cur].xi + KC / 4, buf[cur].xa + KC,
                                           buf[cur].xb + KC, CL::WLEN, wave, rl, h, acc, acc64);
        }
        if constexpr (PATH != HOS_PATH_FP32)   // the FP32 path flushes inside
            flush_acc<NB, true>(acc, acc64, sgn);

        const bool seg_end = !has_next || nq.R != q.R || nq.Cc != q.Cc;
        if (seg_end) {
            const int64_t t = sk_tile_index(q.R, q.Cc);
            double *dst = part + (w * smax + (t - tfirst)) * TILE;
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                bool on;
                int blk;
                if constexpr (PATH == HOS_PATH_FP32) {
                    on = (mask >> cb) & 1;
                    blk = (rowbase + (cb >> 1)) * NB + colbase + (cb & 1);
                } else {
                    on = cb < ncol;
                    blk = wave * NB + cb;
                }
                if (on) {
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        dst[(blk * 16 + v) * 64 + lane] = acc64[cb][v];
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc64[cb][v] = 0.0;
                    if (PATH != HOS_PATH_FP32)
                        pin_agpr(acc64[cb][v]);
                }
            }
        }
        if (!has_next)
            break;
        cur ^= 1;
        if constexpr (!SPLIT)
            store_chunk<PATH, NB, CL::NPW>(stg, buf[cur], wave, lane, nq.c & 1);
        else
            store_xi<CL>(xr, buf[cur], wave, lane, nq.c & 1);
        __syncthreads();
        if (seg_end)
            set_layout(nq);
        q = nq;
    }
}

// tfirst[w] = the tile of workgroup w's first chunk (its slot 0), or -1 for
// a workgroup with no chunk: the same walk the contraction does at its start.
__global__ void __launch_bounds__(256)
k_sk_tfirst(SkGeom g, int64_t *__restrict__ tfirst)
{
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= g.G)
        return;
    SkPos q;
    const int64_t S0 = sk_wg_start(g, w), S1 = sk_wg_start(g, w + 1);
    tfirst[w] = (sk_first_chunk(g, S0, q) && sk_chunk_start(g, q.R, q.Cc, q.c) < S1)
                    ? sk_tile_index(q.R, q.Cc) : -1;
}

// Sum the FP64 partial tiles of every workgroup that touched the tile, in
// workgroup order, and scatter the 32 x 32 block to Cfull[a][b] (a = r + 1).
// One workgroup per (tile, 32-block).
template <int NB>
__global__ void __launch_bounds__(256)
k_c3_reduce(const double *__restrict__ part, const int64_t *__restrict__ tfirst, SkGeom g,
            int64_t smax, int NBR, int M, int corner, double *__restrict__ cfull)
{
    constexpr int64_t TILE = (int64_t)(32 * NB) * (32 * NB);
    // blockIdx.x = (tile, 32-block, quarter of the block's 1024 elements)
    const int q = blockIdx.x & 3;
    const int64_t t = (blockIdx.x >> 2) / (NB * NB);
    const int blk = (blockIdx.x >> 2) % (NB * NB);
    int R = 0;
    while (sk_tile_index(R + 1, 0) <= t)
        ++R;
    const int Cc = (int)(t - sk_tile_index(R, 0));
    const int bR = blk / NB, bC = blk % NB;
    const int Rg = R * NB + bR, Bg = Cc * NB + bC;
    if (Rg >= NBR || Bg > Rg)
        return;
    const int e = threadIdx.x + 256 * q;
    const int64_t w_lo = sk_owner(g, sk_chunk_start(g, R, Cc, 0));
    const int64_t w_hi = sk_owner(g, sk_chunk_start(g, R, Cc, g.C - 1));
    double sum = 0.0;
    // unrolled so the loads go out ahead; the adds keep their order
#pragma unroll 8
    for (int64_t w = w_lo; w <= w_hi; ++w) {
        const int64_t slot = w * smax + (t - tfirst[w]);
        sum += part[slot * TILE + (int64_t)blk * 1024 + e];
    }
    const int v = e >> 6, lane = e & 63;
    // 32x32 MFMA accumulator layout: column = lane % 32,
    // row = 8 (v / 4) + 4 (lane / 32) + v % 4
    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int col = lane & 31;
    const int r = Rg * 32 + row, b = Bg * 32 + col;
    if (!corner) {
        // F: C[r+1][b] for b <= r + 1
        if (r < M && (Bg < Rg || col <= row + 1))
            cfull[(int64_t)(r + 1) * (M + 1) + b] = sum;
    } else {
        // corners: column b is the offset M + 1 + b, so the sum is C[M+1+b][r+1],
        // a lag of the square iff (M + 1 + b) - (r + 1) <= M, i.e. b <= r; it
        // goes to the table's upper triangle at [b][r+1]
        if (r < M && (Bg < Rg || col <= row))
            cfull[(int64_t)b * (M + 1) + (r + 1)] = sum;
    }
}

// Leftover diagonal sums C[a][a] = sum_i x~_i x~_{i+a}^2 for a = 0 and
// a = 32k <= M, in FP64 from the input itself (x~ = (x - mean) s formed in
// FP64, not the FP32 operand copy), as fixed-order partials.
// The first factor x_i runs over i < nfirst only (a piece of a record with
// its halo: nfirst is the piece's own length; n for a whole record).
template <typename T>
__global__ void __launch_bounds__(256)
k_diag_dot(const T *__restrict__ x, int64_t n, const double *__restrict__ stats,
           int nblocks, double *__restrict__ dpart, int64_t nfirst)
{
    __shared__ double red[256];
    const int left = blockIdx.x / nblocks, blk = blockIdx.x % nblocks;
    const int64_t a = 32 * (int64_t)left;
    const double mu = stats[0], sc = stats[1];
    double s = 0.0;
    for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i + a < n && i < nfirst;
         i += (int64_t)nblocks * 256) {
        const double u = ((double)x[i + a] - mu) * sc;
        s += (((double)x[i] - mu) * sc) * u * u;
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

// The same sums for nleft <= DIAG_FUSED_MAX leftovers in one pass over x.
// Workgroup c takes the 2048-sample blocks c, c + gridDim.x, ...: it stages
// x~ (FP64, 0 past n) for the block plus the 32 (nleft - 1) halo in LDS while
// the next block's loads are in flight, and each thread accumulates every
// leftover's products for its consecutive sample pairs (one 16-byte LDS read
// per pair and leftover; the first factor is 0 from nfirst on).  Waves
// reduce by lane shuffles, then the 4 wave sums are added in order:
// dpart[left * gridDim.x + c].  MAXL bounds nleft.
constexpr int DIAG_FUSED_MAX = 32;
constexpr int DF_BLK = 2048;
constexpr int DF_MAX_WG = 256;

template <typename T, int MAXL>
__global__ void __launch_bounds__(256)
k_diag_fused(const T *__restrict__ x, int64_t n, const double *__restrict__ stats, int nleft,
             double *__restrict__ dpart, int64_t nfirst)
{
    constexpr int STAGE = DF_BLK + 32 * (MAXL - 1);
    constexpr int LB = (STAGE + 255) / 256;
    __shared__ __attribute__((aligned(16))) double sx[STAGE];   // read as double2
    __shared__ double wsum[4][MAXL];
    const double mu = stats[0], sc = stats[1];
    const int live = DF_BLK + 32 * (nleft - 1);
    const int64_t step = (int64_t)gridDim.x * DF_BLK;
    double acc[MAXL];
#pragma unroll
    for (int k = 0; k < MAXL; ++k)
        acc[k] = 0.0;
    T v[LB];
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int64_t i = i0 + threadIdx.x + 256 * u;
            v[u] = x[i < n ? i : 0];
        }
    };
    int64_t i0 = (int64_t)blockIdx.x * DF_BLK;
    if (i0 < n)
        fetch(i0);
    for (; i0 < n; i0 += step) {
        __syncthreads();   // the previous block's reads are done
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < live)
                sx[e] = i0 + e < n ? ((double)v[u] - mu) * sc : 0.0;
        }
        __syncthreads();
        if (i0 + step < n)
            fetch(i0 + step);   // in flight during this block's sums
#pragma unroll
        for (int q = 0; q < DF_BLK / 512; ++q) {
            const int j = 2 * threadIdx.x + 512 * q;
            double2 xi = *(const double2 *)&sx[j];
            if (i0 + j >= nfirst)
                xi.x = 0.0;
            if (i0 + j + 1 >= nfirst)
                xi.y = 0.0;
#pragma unroll
            for (int k = 0; k < MAXL; ++k)
                if (k < nleft) {
                    const double2 u = *(const double2 *)&sx[j + 32 * k];
                    acc[k] += xi.x * u.x * u.x;
                    acc[k] += xi.y * u.y * u.y;
                }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < MAXL; ++k) {
        if (k < nleft) {
            double t = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                t += __shfl_xor(t, off, 64);
            if (lane == 0)
                wsum[wv][k] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nleft) {
        const int k = threadIdx.x;
        dpart[k * gridDim.x + blockIdx.x] = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
    }
}

// Workgroups of k_diag_fused for n samples (the plan's dot_blocks = ceil(n /
// 1024) slots per leftover hold them).
inline int diag_fused_grid(int64_t n)
{
    const int64_t b = (n + DF_BLK - 1) / DF_BLK;
    return (int)(b < 1 ? 1 : (b > DF_MAX_WG ? DF_MAX_WG : b));
}

// C[a][a] = the leftover's block partials summed in block order (strided over
// 256 threads, then a fixed tree).  One workgroup per leftover.
__global__ void __launch_bounds__(256)
k_diag_final(const double *__restrict__ dpart, int nleft, int nblocks, int M,
             double *__restrict__ cfull)
{
    __shared__ double red[256];
    const int left = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256)
        s += dpart[left * nblocks + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t a = 32 * (int64_t)left;
        cfull[a * (M + 1) + a] = red[0];
    }
}

// ------------------------------------------------------------------ batches
// The persistent contraction over a batch: workgroup w runs the work items
// wgfirst[w] .. wgfirst[w+1]-1 of the plan (each a chunk range of one tile
// of one series) with the same per-chunk pipeline as k_c3_contract; the
// next chunk, possibly of the next item and another series, is prefetched
// while the current one is computed.  Each item writes its own partial tile.
struct SeriesPtrs {
    const float *xf;
    const uint4 *w4, *w8h, *w8l;
    int NBR;
};

__device__ inline SeriesPtrs series_ptrs(const SeriesDesc &d, const char *ws)
{
    const char *r = ws + d.ws_off;
    SeriesPtrs p;
    p.xf = (const float *)(r + d.o_xf);
    p.w4 = (const uint4 *)(r + d.o_win4);
    p.w8h = (const uint4 *)(r + d.o_win8h);
    p.w8l = (const uint4 *)(r + d.o_win8l);
    p.NBR = d.NBR;
    return p;
}

template <int PATH, int NB>
__global__ void __launch_bounds__(64 * NB, 1)
k_c3_items(const SeriesDesc *__restrict__ sd, const C3Item *__restrict__ items,
           const int32_t *__restrict__ wgfirst, const char *__restrict__ ws,
           double *__restrict__ part)
{
    constexpr bool SPLIT = PATH != HOS_PATH_FP32;
    constexpr int KCX = c3_stage_len(PATH, NB);   // as in k_c3_contract
    typedef ChunkLds<PATH, NB, KCX> CL;
    constexpr int64_t TILE = (int64_t)CL::TS * CL::TS;

    __shared__ CL buf[2];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, rl = lane & 31, h = lane >> 5;
    const int k1 = wgfirst[blockIdx.x + 1];
    int k = wgfirst[blockIdx.x];
    if (k >= k1)
        return;

    C3Item it = items[k];
    SeriesPtrs sp = series_ptrs(sd[it.series], ws);
    SkPos q;
    q.R = it.R;
    q.Cc = it.Cc;
    q.c = it.c0;

    floatx16 acc[NB];
    double acc64[NB][16];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc[cb][v] = 0.0f;
            acc64[cb][v] = 0.0;
            if (PATH != HOS_PATH_FP32)
                pin_agpr(acc64[cb][v]);
        }

    int ncol = 0, rowbase = 0, colbase = 0, mask = 0;
    auto set_layout = [&](const SkPos &p, int NBR) {
        if constexpr (PATH == HOS_PATH_FP32) {
            fp32_window(p.Cc == p.R, wave, p.R, NBR, rowbase, colbase, mask);
            mask = __builtin_amdgcn_readfirstlane(mask);
            rowbase = __builtin_amdgcn_readfirstlane(rowbase);
            colbase = __builtin_amdgcn_readfirstlane(colbase);
        } else {
            ncol = __builtin_amdgcn_readfirstlane(wave_cols(NB, p.Cc == p.R, wave, p.R, NBR));
        }
    };
    set_layout(q, sp.NBR);

    u32x4 stg[CL::NPW];
    XiRegs<CL> xr;
    if constexpr (!SPLIT) {
        load_chunk<PATH, NB, CL::NPW>(stg, sp.xf, sp.w4, sp.w8h, sp.w8l, q, wave, lane, 0);
        store_chunk<PATH, NB, CL::NPW>(stg, buf[0], wave, lane, q.c & 1);
    } else {
        load_chunk_dma<CL>(xr, sp.xf, sp.w4, sp.w8h, sp.w8l, q, buf[0], wave, lane,
                                      0);
        store_xi<CL>(xr, buf[0], wave, lane, q.c & 1);
    }
    __syncthreads();

    int cur = 0;
    for (;;) {
        // the next chunk: the same item, else the first chunk of the next item
        SkPos nq = q;
        C3Item nit = it;
        SeriesPtrs nsp = sp;
        bool has_next = true, new_item = false;
        if (q.c + 1 < it.c1) {
            nq.c = q.c + 1;
        } else if (k + 1 < k1) {
            nit = items[k + 1];
            nsp = series_ptrs(sd[nit.series], ws);
            nq.R = nit.R;
            nq.Cc = nit.Cc;
            nq.c = nit.c0;
            new_item = true;
        } else {
            has_next = false;
        }
        if (has_next) {
            if constexpr (!SPLIT)
                load_chunk<PATH, NB, CL::NPW>(stg, nsp.xf, nsp.w4, nsp.w8h, nsp.w8l, nq, wave,
                                              lane, 0);
            else
                load_chunk_dma<CL>(xr, nsp.xf, nsp.w4, nsp.w8h, nsp.w8l, nq,
                                              buf[cur ^ 1], wave, lane, 0);
        }

        const float sgn = (q.c & 1) ? -1.0f : 1.0f;
        if constexpr (PATH == HOS_PATH_FP32) {
            dispatch_fp32(mask, buf[cur].xi, buf[cur].xa, buf[cur].xb, rowbase, colbase, rl, h,
                          acc, acc64, sgn);
        } else {
            dispatch_compute<PATH, NB>(ncol, buf[cur].xi, buf[cur].xa, buf[cur].xb, CL::WLEN,
                                       wave, rl, h, acc, acc64);
            if constexpr (KCX == 2 * KC)
                dispatch_compute<PATH, NB>(ncol, buf[cur].xi + KC / 4, buf[cur].xa + KC,
                                           buf[cur].xb + KC, CL::WLEN, wave, rl, h, acc, acc64);
        }
        if constexpr (PATH != HOS_PATH_FP32)
            flush_acc<NB, true>(acc, acc64, sgn);

        if (!has_next || new_item) {
            double *dst = part + it.slot * TILE;
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                bool on;
                int blk;
                if constexpr (PATH == HOS_PATH_FP32) {
                    on = (mask >> cb) & 1;
                    blk = (rowbase + (cb >> 1)) * NB + colbase + (cb & 1);
                } else {
                    on = cb < ncol;
                    blk = wave * NB + cb;
                }
                if (on) {
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        dst[(blk * 16 + v) * 64 + lane] = acc64[cb][v];
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc64[cb][v] = 0.0;
                    if (PATH != HOS_PATH_FP32)
                        pin_agpr(acc64[cb][v]);
                }
            }
        }
        if (!has_next)
            break;
        cur ^= 1;
        if constexpr (!SPLIT)
            store_chunk<PATH, NB, CL::NPW>(stg, buf[cur], wave, lane, nq.c & 1);
        else
            store_xi<CL>(xr, buf[cur], wave, lane, nq.c & 1);
        __syncthreads();
        if (new_item) {
            ++k;
            it = nit;
            sp = nsp;
            set_layout(nq, sp.NBR);
        }
        q = nq;
    }
}

// The batch contraction of the split paths in ONE persistent launch over
// both tile classes.  Workgroups have 4 waves and stage 1024-sample chunks
// (as k_c3_contract's 4-block tiles).  On an item of 4 x 4 blocks wave w
// owns strip w.  On an item of 2 x 2 blocks the waves w and w + 2 share
// strip w & 1: wave w < 2 computes the first 512 samples of every chunk and
// wave w + 2 the second 512 (a split of the sample axis inside the
// workgroup, so the class runs at the same 4 waves and the same chunk); at
// the item's end waves 2 and 3 hand their FP64 sums over through LDS and
// waves 0 and 1 add them (a fixed order) and write the partial.  A
// workgroup's list (one LPT schedule over both classes) holds its 4 x 4
// items first; each class runs in a loop of its own, so each loop keeps the
// register budget of a one-class kernel.
template <int PATH, int CLS>
__device__ __attribute__((always_inline)) inline void
items_loop(const SeriesDesc *__restrict__ sd, const C3Item *__restrict__ items, int k, int k1,
           const char *__restrict__ ws, double *__restrict__ part, uint4 *lds, int bufsz,
           double *hand, int wave, int lane)
{
    constexpr int NB = CLS ? 4 : 2;
    typedef ChunkLds<PATH, NB, 2 * KC, 4> CL;
    constexpr int64_t TILE = (int64_t)CL::TS * CL::TS;
    const int rl = lane & 31, h = lane >> 5;
    // 2 x 2 items of a series with one 32-row block (M < 33) have no strip
    // 1: the four waves then run strip 0 on the four quarters of the chunk
    // (else the strip-1 waves would idle)
    auto strip_of = [&](int nbr) { return CLS ? wave : (nbr == 1 ? 0 : (wave & 1)); };
    auto buf = [&](int b) -> CL & { return *reinterpret_cast<CL *>(lds + b * bufsz); };

    C3Item it = items[k];
    SeriesPtrs sp = series_ptrs(sd[it.series], ws);
    SkPos q;
    q.R = it.R;
    q.Cc = it.Cc;
    q.c = it.c0;

    floatx16 acc[NB];
    double acc64[NB][16];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc[cb][v] = 0.0f;
            acc64[cb][v] = 0.0;
            pin_agpr(acc64[cb][v]);
        }
    int strip = strip_of(sp.NBR);
    int ncol = __builtin_amdgcn_readfirstlane(wave_cols(NB, q.Cc == q.R, strip, q.R, sp.NBR));

    XiRegs<CL> xr;
    load_chunk_dma<CL>(xr, sp.xf, sp.w4, sp.w8h, sp.w8l, q, buf(0), wave, lane, 0);
    store_xi<CL>(xr, buf(0), wave, lane, q.c & 1);
    __syncthreads();

    int cur = 0;
    for (;;) {
        SkPos nq = q;
        C3Item nit = it;
        SeriesPtrs nsp = sp;
        bool has_next = true, new_item = false;
        if (q.c + 1 < it.c1) {
            nq.c = q.c + 1;
        } else if (k + 1 < k1) {
            nit = items[k + 1];
            nsp = series_ptrs(sd[nit.series], ws);
            nq.R = nit.R;
            nq.Cc = nit.Cc;
            nq.c = nit.c0;
            new_item = true;
        } else {
            has_next = false;
        }
        if (has_next)
            load_chunk_dma<CL>(xr, nsp.xf, nsp.w4, nsp.w8h, nsp.w8l, nq, buf(cur ^ 1), wave,
                               lane, 0);

        const float sgn = (q.c & 1) ? -1.0f : 1.0f;
        CL &B = buf(cur);
        if constexpr (CLS) {
            dispatch_compute<PATH, 4>(ncol, B.xi, B.xa, B.xb, CL::WLEN, strip, rl, h, acc, acc64);
            dispatch_compute<PATH, 4>(ncol, B.xi + KC / 4, B.xa + KC, B.xb + KC, CL::WLEN, strip,
                                      rl, h, acc, acc64);
        } else if (sp.NBR == 1) {
            const int o = wave * (KC / 2);   // this wave's quarter of the chunk
            dispatch_compute<PATH, 2, 2, KC / GROUP / 2>(ncol, B.xi + o / 4, B.xa + o, B.xb + o,
                                                         CL::WLEN, 0, rl, h, acc, acc64);
        } else {
            const int o = (wave >> 1) * KC;   // this wave's half of the chunk
            dispatch_compute<PATH, 2>(ncol, B.xi + o / 4, B.xa + o, B.xb + o, CL::WLEN, strip,
                                      rl, h, acc, acc64);
        }
        flush_acc<NB, true>(acc, acc64, sgn);

        if (!has_next || new_item) {
            double *dst = part + it.slot * TILE;
            if constexpr (CLS) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    if (cb < ncol) {
#pragma unroll
                        for (int v = 0; v < 16; ++v)
                            dst[((strip * 4 + cb) * 16 + v) * 64 + lane] = acc64[cb][v];
                    }
            } else if (sp.NBR == 1) {
                // waves 1-3's quarters to wave 0, in LDS, added in wave order
                if (wave >= 1) {
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        hand[((wave - 1) * 16 + v) * 64 + lane] = acc64[0][v];
                }
                __syncthreads();
                if (wave == 0) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int e = v * 64 + lane;
                        dst[e] = ((acc64[0][v] + hand[e]) + hand[1024 + e]) + hand[2048 + e];
                    }
                }
            } else {
                // the second half's sums to the first half's waves, in LDS
                if (wave >= 2) {
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int v = 0; v < 16; ++v)
                            hand[((strip * 2 + cb) * 16 + v) * 64 + lane] = acc64[cb][v];
                }
                __syncthreads();
                if (wave < 2) {
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        if (cb < ncol) {
#pragma unroll
                            for (int v = 0; v < 16; ++v) {
                                const int e = ((strip * 2 + cb) * 16 + v) * 64 + lane;
                                dst[e] = acc64[cb][v] + hand[e];
                            }
                        }
                }
            }
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc64[cb][v] = 0.0;
                    pin_agpr(acc64[cb][v]);
                }
        }
        if (!has_next)
            break;
        cur ^= 1;
        store_xi<CL>(xr, buf(cur), wave, lane, nq.c & 1);
        __syncthreads();
        if (new_item) {
            ++k;
            it = nit;
            sp = nsp;
            strip = strip_of(sp.NBR);
            ncol = __builtin_amdgcn_readfirstlane(
                wave_cols(NB, nq.Cc == nq.R, strip, nq.R, sp.NBR));
        }
        q = nq;
    }
}

template <int PATH>
__global__ void __launch_bounds__(256, 1)
k_c3_items_u(const SeriesDesc *__restrict__ sd, const C3Item *__restrict__ items,
             const int32_t *__restrict__ wgfirst, const char *__restrict__ ws,
             double *__restrict__ part2, double *__restrict__ part4)
{
    static_assert(PATH != HOS_PATH_FP32, "the FP32 path has one tile class");
    typedef ChunkLds<PATH, 4, 2 * KC, 4> CL4;
    typedef ChunkLds<PATH, 2, 2 * KC, 4> CL2;
    constexpr int BUF = (int)((sizeof(CL4) > sizeof(CL2) ? sizeof(CL4) : sizeof(CL2)) / 16);
    constexpr int HAND = 2 * 2 * 16 * 64 / 2;   // waves 2, 3: 2 blocks x 16 x 64 doubles

    __shared__ uint4 lds[2 * BUF + HAND];
    double *hand = (double *)(lds + 2 * BUF);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k0 = wgfirst[blockIdx.x], k1 = wgfirst[blockIdx.x + 1];
    int mid = k0;   // the 4 x 4 items come first
    while (mid < k1 && items[mid].pad == 1)
        ++mid;
    if (k0 < mid)
        items_loop<PATH, 1>(sd, items, k0, mid, ws, part4, lds, BUF, hand, wave, lane);
    if (mid < k1) {
        if (k0 < mid)
            __syncthreads();   // the first loop's last reads of the buffers are done
        items_loop<PATH, 0>(sd, items, mid, k1, ws, part2, lds, BUF, hand, wave, lane);
    }
}

// Sum the slots of one (series, tile) in order and scatter one 32 x 32 block
// into the series' C[a][b] table.  One workgroup per (tile, block), each
// thread four elements of it: the four loads of a slot go out together and
// each element's slots are added in slot order.
template <int NB>
__global__ void __launch_bounds__(256)
k_c3_reduce_items(const SeriesDesc *__restrict__ sd, const C3TileRef *__restrict__ tiles,
                  const double *__restrict__ part, char *__restrict__ ws)
{
    constexpr int64_t TILE = (int64_t)(32 * NB) * (32 * NB);
    const C3TileRef t = tiles[blockIdx.x / (NB * NB)];
    const int blk = blockIdx.x % (NB * NB);
    const SeriesDesc &d = sd[t.series];
    const int bR = blk / NB, bC = blk % NB;
    const int Rg = t.R * NB + bR, Bg = t.Cc * NB + bC;
    if (Rg >= d.NBR || Bg > Rg)
        return;
    const int M = d.M;
    double *cfull = (double *)(ws + d.ws_off + d.o_cfull);
    const double *src = part + t.slot0 * TILE + (int64_t)blk * 1024 + threadIdx.x;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int j = 0; j < t.nslot; ++j) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = src[j * TILE + 256 * q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            sum[q] += v[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int v = e >> 6, lane = e & 63;
        const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = lane & 31;
        const int r = Rg * 32 + row, b = Bg * 32 + col;
        if (r < M && (Bg < Rg || col <= row + 1))
            cfull[(int64_t)(r + 1) * (M + 1) + b] = sum[q];
    }
}

// Leftover diagonal sums C[a][a] = sum_i x~_i x~_{i+a}^2, a = 32 k <= M,
// in FP64 from the input.  Workgroup (c, s) takes the BD_BLK-sample blocks
// c, c + nchunk, ... of series s: their centred, scaled samples x~ (plus the
// 32 (nleft - 1) halo) pass through LDS, formed once per sample, while the
// next block's loads are already in flight; each thread takes consecutive
// sample pairs (one 16-byte LDS read per pair and diagonal) and accumulates
// every diagonal of the series.  A fixed-order reduction per diagonal (wave
// butterfly, then the four waves in order) leaves the chunk's partial in
// dpart[k nchunk + c]; k_bdiag_final sums the chunks in order.  x~ is 0 past
// the series' end.  MAXL bounds nleft = 1 + M / 32.
constexpr int BD_BLK = 2048;
constexpr int BD_MAXLEFT = 33;   // 1 + M / 32 for M <= 1024

template <typename T, int MAXL>
__global__ void __launch_bounds__(256)
k_bdiag(const T *__restrict__ x, const SeriesDesc *__restrict__ sd, char *__restrict__ ws,
        int nchunk)
{
    constexpr int STAGE = BD_BLK + 32 * (MAXL - 1);
    constexpr int LB = (STAGE + 255) / 256;
    __shared__ __attribute__((aligned(16))) double sx[STAGE];   // read as double2
    __shared__ double wsum[4][MAXL];
    const SeriesDesc &d = sd[blockIdx.y];
    const int nleft = d.nleft, c = blockIdx.x;
    char *r = ws + d.ws_off;
    const double *stats = (const double *)(r + d.o_stats);
    const T *xs = x + d.x_off;
    const int64_t n = d.n;
    const double mu = stats[0], sc = stats[1];
    const int live = BD_BLK + 32 * (nleft - 1);   // staged samples per block
    double acc[MAXL];
#pragma unroll
    for (int k = 0; k < MAXL; ++k)
        acc[k] = 0.0;
    T v[LB];
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int64_t i = i0 + threadIdx.x + 256 * u;
            v[u] = xs[i < n ? i : 0];
        }
    };
    int64_t i0 = (int64_t)c * BD_BLK;
    if (i0 < n)
        fetch(i0);
    for (; i0 < n; i0 += (int64_t)nchunk * BD_BLK) {
        __syncthreads();   // the previous block's reads are done
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < live)
                sx[e] = i0 + e < n ? ((double)v[u] - mu) * sc : 0.0;
        }
        __syncthreads();
        const int64_t next = i0 + (int64_t)nchunk * BD_BLK;
        if (next < n)
            fetch(next);   // in flight during this block's sums
#pragma unroll
        for (int q = 0; q < BD_BLK / 512; ++q) {
            const int j = 2 * threadIdx.x + 512 * q;
            const double2 xi = *(const double2 *)&sx[j];
#pragma unroll
            for (int k = 0; k < MAXL; ++k)
                if (k < nleft) {
                    const double2 u = *(const double2 *)&sx[j + 32 * k];
                    acc[k] += xi.x * u.x * u.x;
                    acc[k] += xi.y * u.y * u.y;
                }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < MAXL; ++k) {
        if (k < nleft) {
            double t = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                t += __shfl_xor(t, off, 64);
            if (lane == 0)
                wsum[wv][k] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nleft) {
        const int k = threadIdx.x;
        ((double *)(r + d.o_dpart))[k * nchunk + c] =
            ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
    }
}

// C[a][a], a = 32 k: the chunk partials of diagonal k summed in chunk order.
__global__ void __launch_bounds__(64)
k_bdiag_final(const SeriesDesc *__restrict__ sd, char *__restrict__ ws, int nchunk)
{
    const SeriesDesc &d = sd[blockIdx.x];
    char *r = ws + d.ws_off;
    const double *dpart = (const double *)(r + d.o_dpart);
    for (int k = threadIdx.x; k < d.nleft; k += 64) {
        double t = 0.0;
        for (int c = 0; c < nchunk; ++c)
            t += dpart[k * nchunk + c];
        const int64_t a = 32 * (int64_t)k;
        ((double *)(r + d.o_cfull))[a * (d.M + 1) + a] = t;
    }
}

template <typename T>
void launch_bdiag_t(const T *x, const BatchHeader &h, const SeriesDesc *sd, char *ws,
                    hipStream_t s)
{
    // enough chunks per series for about 2048 workgroups in all, at most the
    // dot_blocks slots the plan gave each diagonal
    int64_t nchunk = (2048 + h.batch - 1) / h.batch;
    if (nchunk > h.dot_blocks)
        nchunk = h.dot_blocks;
    if (nchunk < 1)
        nchunk = 1;
    const dim3 grid((unsigned)nchunk, (unsigned)h.batch);
    if (h.max_nleft <= 9)
        k_bdiag<T, 9><<<grid, 256, 0, s>>>(x, sd, ws, (int)nchunk);
    else if (h.max_nleft <= 17)
        k_bdiag<T, 17><<<grid, 256, 0, s>>>(x, sd, ws, (int)nchunk);
    else
        k_bdiag<T, BD_MAXLEFT><<<grid, 256, 0, s>>>(x, sd, ws, (int)nchunk);
    k_bdiag_final<<<(unsigned)h.batch, 64, 0, s>>>(sd, ws, (int)nchunk);
}

// FP32 path: one tile class (4 x 4 blocks), the generic per-class kernel.
void launch_items_fp32(const BatchHeader &h, const char *dplan, char *ws, hipStream_t s)
{
    k_c3_items<HOS_PATH_FP32, 4><<<(unsigned)h.G[1], 256, 0, s>>>(
        (const SeriesDesc *)(dplan + h.series_off), (const C3Item *)(dplan + h.items_off),
        (const int32_t *)(dplan + h.wgfirst_off), ws, (double *)(ws + h.part_off[1]));
}

// Split paths: both classes in one launch.
template <int PATH>
void launch_items_u(const BatchHeader &h, const char *dplan, char *ws, hipStream_t s)
{
    k_c3_items_u<PATH><<<(unsigned)h.G[0], 256, 0, s>>>(
        (const SeriesDesc *)(dplan + h.series_off), (const C3Item *)(dplan + h.items_off),
        (const int32_t *)(dplan + h.wgfirst_off), ws, (double *)(ws + h.part_off[0]),
        (double *)(ws + h.part_off[1]));
}

template <int PATH, int NB>
void launch_contract_t(const C3Plan &p, char *ws, hipStream_t s, int64_t coff)
{
    k_c3_contract<PATH, NB><<<p.sk.G, 64 * NB, 0, s>>>(
        (const float *)(ws + p.off_xf), (const uint4 *)(ws + p.off_win4),
        (const uint4 *)(ws + p.off_win8h), (const uint4 *)(ws + p.off_win8l),
        (double *)(ws + p.off_part), p.sk, p.smax, p.NBR, coff);
}

}  // namespace

hipError_t launch_c3_contract(const C3Plan &p, char *ws, hipStream_t s, int region)
{
    if (region == 1 && p.amax <= p.M)
        return hipErrorInvalidValue;   // the plan has no corner rows
    const int64_t coff = region == 1 ? (int64_t)p.M + 1 : 0;
    if (p.M > 0) {
        if (p.NB == 4) {
            if (p.path == HOS_PATH_FP32)
                launch_contract_t<HOS_PATH_FP32, 4>(p, ws, s, coff);
            else if (p.path == HOS_PATH_SPLIT_FP16)
                launch_contract_t<HOS_PATH_SPLIT_FP16, 4>(p, ws, s, coff);
            else
                launch_contract_t<HOS_PATH_SPLIT_BF16, 4>(p, ws, s, coff);
        } else {
            if (p.path == HOS_PATH_SPLIT_FP16)
                launch_contract_t<HOS_PATH_SPLIT_FP16, 2>(p, ws, s, coff);
            else
                launch_contract_t<HOS_PATH_SPLIT_BF16, 2>(p, ws, s, coff);
        }
    }
    return hipGetLastError();
}

hipError_t launch_diag_dot(const void *x, int dtype, const C3Plan &p, char *ws, hipStream_t s,
                           int64_t nfirst)
{
    const double *stats = (const double *)(ws + p.off_stats);
    double *dpart = (double *)(ws + p.off_dpart);
    if (nfirst < 0)
        nfirst = p.n;
    if (p.nleft <= DIAG_FUSED_MAX) {   // the plan made dot_blocks = ceil(n / 1024)
        const int g = diag_fused_grid(p.n);
#define HOS_DIAG_FUSED(T, L)                                                              \
    k_diag_fused<T, L><<<g, 256, 0, s>>>((const T *)x, p.n, stats, p.nleft, dpart, nfirst)
        if (dtype == HOS_F64) {
            if (p.nleft <= 9)
                HOS_DIAG_FUSED(double, 9);
            else if (p.nleft <= 17)
                HOS_DIAG_FUSED(double, 17);
            else
                HOS_DIAG_FUSED(double, DIAG_FUSED_MAX);
        } else {
            if (p.nleft <= 9)
                HOS_DIAG_FUSED(float, 9);
            else if (p.nleft <= 17)
                HOS_DIAG_FUSED(float, 17);
            else
                HOS_DIAG_FUSED(float, DIAG_FUSED_MAX);
        }
#undef HOS_DIAG_FUSED
        return hipGetLastError();
    }
    const int grid = p.nleft * p.dot_blocks;
    if (dtype == HOS_F64)
        k_diag_dot<double><<<grid, 256, 0, s>>>((const double *)x, p.n, stats, p.dot_blocks, dpart,
                                                nfirst);
    else
        k_diag_dot<float><<<grid, 256, 0, s>>>((const float *)x, p.n, stats, p.dot_blocks, dpart,
                                               nfirst);
    return hipGetLastError();
}

hipError_t launch_c3_reduce(const C3Plan &p, char *ws, hipStream_t s, int region)
{
    if (region == 1 && p.amax <= p.M)
        return hipErrorInvalidValue;
    double *cfull = (double *)(ws + p.off_cfull);
    if (p.M > 0) {
        const int64_t ntiles = (int64_t)p.sk.TR * (p.sk.TR + 1) / 2;
        const int NB = p.NB;
        k_sk_tfirst<<<(p.sk.G + 255) / 256, 256, 0, s>>>(p.sk, (int64_t *)(ws + p.off_tfirst));
        if (NB == 4)
            k_c3_reduce<4><<<ntiles * NB * NB * 4, 256, 0, s>>>(
                (const double *)(ws + p.off_part), (const int64_t *)(ws + p.off_tfirst), p.sk,
                p.smax, p.NBR, p.M, region, cfull);
        else
            k_c3_reduce<2><<<ntiles * NB * NB * 4, 256, 0, s>>>(
                (const double *)(ws + p.off_part), (const int64_t *)(ws + p.off_tfirst), p.sk,
                p.smax, p.NBR, p.M, region, cfull);
    }
    if (region == 0)   // the diagonal sums C[a][a], a = 0 and a = 32k, belong to F
        k_diag_final<<<p.nleft, 256, 0, s>>>(
            (const double *)(ws + p.off_dpart), p.nleft,
            p.nleft <= DIAG_FUSED_MAX ? diag_fused_grid(p.n) : p.dot_blocks, p.M, cfull);
    return hipGetLastError();
}

}  // namespace hos

namespace hos {

// One persistent launch over every work item of the batch.
hipError_t launch_batch_contract(const BatchHeader &h, const char *dplan, char *ws,
                                 hipStream_t s)
{
    if (h.n_items_all == 0)
        return hipGetLastError();
    if (h.path == HOS_PATH_FP32)
        launch_items_fp32(h, dplan, ws, s);
    else if (h.path == HOS_PATH_SPLIT_FP16)
        launch_items_u<HOS_PATH_SPLIT_FP16>(h, dplan, ws, s);
    else
        launch_items_u<HOS_PATH_SPLIT_BF16>(h, dplan, ws, s);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const void *x, int dtype, const BatchHeader &h, const char *dplan,
                               char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    for (int cls = 0; cls < BATCH_CLASSES; ++cls) {
        if (h.n_tiles[cls] == 0)
            continue;
        const C3TileRef *t = (const C3TileRef *)(dplan + h.tiles_off[cls]);
        const double *part = (const double *)(ws + h.part_off[cls]);
        if (cls == 1)
            k_c3_reduce_items<4><<<(unsigned)(h.n_tiles[cls] * 16), 256, 0, s>>>(sd, t, part, ws);
        else
            k_c3_reduce_items<2><<<(unsigned)(h.n_tiles[cls] * 4), 256, 0, s>>>(sd, t, part, ws);
    }
    // every leftover diagonal of a series in one pass over its samples
    if (h.max_nleft > BD_MAXLEFT)
        return hipErrorInvalidValue;
    if (dtype == HOS_F64)
        launch_bdiag_t((const double *)x, h, sd, ws, s);
    else
        launch_bdiag_t((const float *)x, h, sd, ws, s);
    return hipGetLastError();
}

}  // namespace hos
