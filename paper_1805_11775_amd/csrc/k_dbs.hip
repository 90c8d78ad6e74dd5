// k_dbs.hip -- the direct bispectrum method (Algorithm DBS) with the
// window-sum smoothing of Section 3 (Algorithm WS and its 2-D form).
//
// The series is cut into K parts of P samples (trailing samples unused),
// each part loses its own FP64 mean and gets a P-point DFT F_i.  The raw
// bispectrum F_i(k1) F_i(k2) conj F_i(k1 + k2) / P, the M3 x M3 box average
// and the average over parts are all linear, so
// the parts are summed first and the sum is smoothed once:
//     B(k1, k2) = 1 / (K P M3^2) sum_{q, c in box} sum_i F_i(q) F_i(c) conj F_i(q + c),
// the box being q in [k1 - lo, k1 + hi], c in [k2 - lo, k2 + hi],
// lo = floor(M3 / 2), hi = M3 - 1 - lo, every index taken modulo P.
//
// The box sum is separable.  Each workgroup owns a strip of TW output
// columns and a run of output rows.  Row by row it forms the products of
// the strip widened by the box (W = TW + M3 - 1 columns), turns them into
// window sums along k2 with one prefix scan (the 1-D window sum as a
// difference of two prefix sums), and keeps a sliding window sum down each
// column: the entering row is added and the row leaving the box is formed
// again and subtracted (the 1-D recurrence s_{i+1} = s_i - k_i + k_{i+j}).
// Every output therefore costs O(1) work whatever M3, and nothing but the
// principal-domain outputs is written to memory.
//
// K = 1: products are formed from the spectrum, with F(q) taken out of the
// row sum.  K >= 2: the part sums are formed first on the rectangle the
// strips read (k_dbs_rawsum, FP64 register tiles over the parts, in part
// groups reduced in a fixed order), and the smoothing reads them.
#include "hos_internal.h"
#include "hos_fft.h"

namespace hos {

namespace {

constexpr int MEAN_SPAN = 2048;   // samples per mean workgroup (8 per thread)

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

__device__ inline int wrap_p(int64_t v, int P)
{
    int64_t r = v % P;
    return (int)(r < 0 ? r + P : r);
}

__device__ inline double2 shfl_up2(double2 v, int d)
{
    return make_double2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}

// Offset of row k1 of the principal domain 0 <= k2 <= k1, k1 + k2 <= H
// (row k1 holds min(k1, H - k1) + 1 points).
__device__ inline int64_t pd_row_off(int r, int H)
{
    const int64_t m = H / 2;
    auto tri = [](int64_t t) { return t * (t + 1) / 2; };
    if (r <= m + 1)
        return tri(r);
    return tri(m + 1) + tri(H - m) - tri((int64_t)H + 1 - r);
}

// Per-part mean removal: partial sums of each part, MEAN_SPAN samples per workgroup.
template <typename T>
__global__ void __launch_bounds__(256)
k_dbs_psum(const T *__restrict__ x, int P, int bpp, double *__restrict__ psum)
{
    __shared__ double red[256];
    const int64_t part = blockIdx.x / bpp;
    const int b = blockIdx.x - (int)part * bpp;
    const T *xp = x + part * P;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < MEAN_SPAN / 256; ++k) {
        const int u = b * MEAN_SPAN + k * 256 + threadIdx.x;
        if (u < P)
            s += (double)xp[u];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        psum[blockIdx.x] = red[0];
}

__device__ inline double part_mean(const double *__restrict__ psum, int64_t part, int bpp,
                                   int P, bool center)
{
    if (!center)
        return 0.0;
    double s = 0.0;
    for (int b = 0; b < bpp; ++b)
        s += psum[part * bpp + b];
    return s / (double)P;
}

// Part DFT, P <= DBS_LDS_FFT: CB whole parts per workgroup in LDS.
template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
k_dbs_fft1(const T *__restrict__ x, const double *__restrict__ psum, int bpp, int64_t K,
           FftRadices fr, int CB, const double2 *__restrict__ tw, int center,
           double2 *__restrict__ F)
{
    __shared__ double2 sm[FFT_LDS_ELEMS];
    __shared__ double mu[32];
    const int P = fr.n;
    const int64_t i0 = (int64_t)blockIdx.x * CB;
    if (threadIdx.x < CB && i0 + threadIdx.x < K)
        mu[threadIdx.x] = part_mean(psum, i0 + threadIdx.x, bpp, P, center != 0);
    __syncthreads();
    for (int e = threadIdx.x; e < CB * P; e += FFT_THREADS) {
        const int cb = e / P, u = e - cb * P;
        const int64_t i = i0 + cb;
        sm[e] = i < K ? make_double2((double)x[i * P + u] - mu[cb], 0.0) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    fft_lds(sm, tw, fr, CB);
    for (int e = threadIdx.x; e < CB * P; e += FFT_THREADS) {
        const int cb = e / P;
        const int64_t i = i0 + cb;
        if (i < K)
            F[i * P + (e - cb * P)] = sm[e];
    }
}

// Part DFT, P = P1 * P2 > DBS_LDS_FFT, first pass: with u = P2 n1 + n2 and
// k = k1 + P1 k2, the length-P1 DFTs over n1 for every n2, each output
// multiplied by exp(-2 pi i n2 k1 / P), stored at [k1][n2].
template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
k_dbs_fft_a(const T *__restrict__ x, const double *__restrict__ psum, int bpp, int64_t K,
            int P2, FftRadices fr1, int CB, const double2 *__restrict__ tw1,
            const double2 *__restrict__ twP, int center, double2 *__restrict__ Tb)
{
    __shared__ double2 sm[FFT_LDS_ELEMS];
    __shared__ double mu[32];
    const int P1 = fr1.n, P = P1 * P2;
    const int64_t nseq = K * P2, s0 = (int64_t)blockIdx.x * CB;
    if (threadIdx.x < CB && s0 + threadIdx.x < nseq)
        mu[threadIdx.x] = part_mean(psum, (s0 + threadIdx.x) / P2, bpp, P, center != 0);
    __syncthreads();
    for (int e = threadIdx.x; e < CB * P1; e += FFT_THREADS) {
        const int n1 = e / CB, cb = e - n1 * CB;
        const int64_t s = s0 + cb;
        double v = 0.0;
        if (s < nseq) {
            const int64_t i = s / P2;
            const int n2 = (int)(s - i * P2);
            v = (double)x[i * P + (int64_t)P2 * n1 + n2] - mu[cb];
        }
        sm[cb * P1 + n1] = make_double2(v, 0.0);
    }
    __syncthreads();
    fft_lds(sm, tw1, fr1, CB);
    for (int e = threadIdx.x; e < CB * P1; e += FFT_THREADS) {
        const int k1 = e / CB, cb = e - k1 * CB;
        const int64_t s = s0 + cb;
        if (s < nseq) {
            const int64_t i = s / P2;
            const int n2 = (int)(s - i * P2);
            Tb[i * P + (int64_t)k1 * P2 + n2] = cmul(sm[cb * P1 + k1], twP[n2 * k1]);
        }
    }
}

// Second pass: the length-P2 DFTs over n2 of every row k1, stored in
// natural order F[k1 + P1 k2].
__global__ void __launch_bounds__(FFT_THREADS)
k_dbs_fft_b(const double2 *__restrict__ Tb, int64_t K, int P1, FftRadices fr2, int CB,
            const double2 *__restrict__ tw2, double2 *__restrict__ F)
{
    __shared__ double2 sm[FFT_LDS_ELEMS];
    const int P2 = fr2.n, P = P1 * P2;
    const int64_t nseq = K * P1, s0 = (int64_t)blockIdx.x * CB;
    for (int e = threadIdx.x; e < CB * P2; e += FFT_THREADS) {
        const int cb = e / P2, n2 = e - cb * P2;
        const int64_t s = s0 + cb;
        if (s < nseq) {
            const int64_t i = s / P1;
            const int k1 = (int)(s - i * P1);
            sm[e] = Tb[i * P + (int64_t)k1 * P2 + n2];
        } else {
            sm[e] = make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    fft_lds(sm, tw2, fr2, CB);
    for (int e = threadIdx.x; e < CB * P2; e += FFT_THREADS) {
        const int k2 = e / CB, cb = e - k2 * CB;
        const int64_t s = s0 + cb;
        if (s < nseq) {
            const int64_t i = s / P1;
            const int k1 = (int)(s - i * P1);
            F[i * P + k1 + (int64_t)P1 * k2] = sm[cb * P2 + k2];
        }
    }
}

// K >= 2: part sums S(q, c) = sum_i F_i(q) F_i(c) conj F_i(q + c) on the
// rectangle q in [-lo, SR - lo), c in [-lo, SC - lo), for the parts of
// group blockIdx.z.  64 x 64 points per workgroup, 4 x 4 per thread; each
// part's 64 row values, 64 column values and 127 diagonal values are
// staged in LDS, PB parts at a time.
constexpr int RS_PB = 8;

__global__ void __launch_bounds__(256)
k_dbs_rawsum(const double2 *__restrict__ F, int P, int64_t K, int Kg, int lo, int SR, int SC,
             double2 *__restrict__ S)
{
    __shared__ double2 fr[RS_PB][64], fc[RS_PB][64], fd[RS_PB][128];
    const int q0 = blockIdx.y * 64 - lo, cc0 = blockIdx.x * 64 - lo;
    const int64_t i_lo = (int64_t)blockIdx.z * Kg;
    const int64_t i_hi = min(K, i_lo + Kg);
    const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            acc[a][b] = make_double2(0.0, 0.0);
    for (int64_t ib = i_lo; ib < i_hi; ib += RS_PB) {
        const int np = (int)min((int64_t)RS_PB, i_hi - ib);
        for (int e = t; e < np * 256; e += 256) {
            const int p = e >> 8, k = e & 255;
            const double2 *Fi = F + (ib + p) * P;
            if (k < 64)
                fr[p][k] = Fi[wrap_p((int64_t)q0 + k, P)];
            else if (k < 128)
                fc[p][k - 64] = Fi[wrap_p((int64_t)cc0 + k - 64, P)];
            else
                fd[p][k - 128] = cconj(Fi[wrap_p((int64_t)q0 + cc0 + k - 128, P)]);
        }
        __syncthreads();
        for (int p = 0; p < np; ++p) {
            double2 rr[4], cv[4], dd[7];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                rr[a] = fr[p][ty + 16 * a];
                cv[a] = fc[p][tx + 16 * a];
            }
#pragma unroll
            for (int s = 0; s < 7; ++s)
                dd[s] = fd[p][ty + tx + 16 * s];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double2 u = cmul(rr[a], cv[b]), d = dd[a + b];
                    acc[a][b].x += u.x * d.x - u.y * d.y;
                    acc[a][b].y += u.x * d.y + u.y * d.x;
                }
        }
        __syncthreads();
    }
    double2 *Sg = S + (int64_t)blockIdx.z * SR * SC;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = blockIdx.y * 64 + ty + 16 * a, col = blockIdx.x * 64 + tx + 16 * b;
            if (row < SR && col < SC)
                Sg[(int64_t)row * SC + col] = acc[a][b];
        }
}

// Sum of the G group rectangles into the first, in group order.
__global__ void __launch_bounds__(256)
k_dbs_sreduce(double2 *__restrict__ S, int G, int64_t count)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count)
        return;
    double2 s = S[e];
    for (int g = 1; g < G; ++g)
        s = cadd(s, S[(int64_t)g * count + e]);
    S[e] = s;
}

// 64-lane inclusive scan of a complex double with DPP lane moves: four
// in-row shifts (Hillis-Steele over 16 lanes), then the last lane of rows
// 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3.  Lanes whose
// source is outside the row, or whose row is masked off, receive 0.
// Lane moves of a complex double.  Shifts within rows of 16 lanes write 0
// to the lanes with no source; the row broadcasts leave masked rows at 0.
template <int CTRL>
__device__ inline double dpp_shr(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <int CTRL, int ROWS>
__device__ inline double dpp_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <int CTRL>
__device__ inline double2 shr_c(double2 v)
{
    return make_double2(dpp_shr<CTRL>(v.x), dpp_shr<CTRL>(v.y));
}

template <int CTRL, int ROWS>
__device__ inline double2 bcast_c(double2 v)
{
    return make_double2(dpp_bcast<CTRL, ROWS>(v.x), dpp_bcast<CTRL, ROWS>(v.y));
}

// 64-lane inclusive scan: four in-row shifts (Hillis-Steele over 16
// lanes), then the last lane of rows 0 and 2 into rows 1 and 3, then lane
// 31 into rows 2 and 3.
__device__ inline double2 wave_scan_incl(double2 v)
{
    v = cadd(v, shr_c<0x111>(v));          // row_shr:1
    v = cadd(v, shr_c<0x112>(v));          // row_shr:2
    v = cadd(v, shr_c<0x114>(v));          // row_shr:4
    v = cadd(v, shr_c<0x118>(v));          // row_shr:8
    v = cadd(v, bcast_c<0x142, 0xa>(v));   // row_bcast:15 -> rows 1, 3
    v = cadd(v, bcast_c<0x143, 0xc>(v));   // row_bcast:31 -> rows 2, 3
    return v;
}

__device__ inline int inc_wrap(int i, int P) { return i + 1 == P ? 0 : i + 1; }

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS (and scalar) operations, not for its global loads and stores,
// which stay in flight across it (no value crosses threads through global
// memory in the smoothing kernel).  s_waitcnt 0xc07f = lgkmcnt(0) with the
// vector-memory and export counters left at their maxima.
__device__ inline void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Sum of the totals of the waves before this one (wave is uniform): lane
// l reads the total of wave l mod NW, a short in-row scan forms the
// running sums over lanes 0 .. NW-1, and lane wave - 1 holds the answer.
template <int NW>
__device__ inline double2 waves_before(const double2 *tot, int lane, int wave)
{
    if (wave == 0)
        return make_double2(0.0, 0.0);
    double2 v = tot[lane & (NW - 1)];
    v = cadd(v, shr_c<0x111>(v));
    if constexpr (NW > 2)
        v = cadd(v, shr_c<0x112>(v));
    if constexpr (NW > 4)
        v = cadd(v, shr_c<0x114>(v));
    const int src = wave - 1;
    const long long bx = __double_as_longlong(v.x), by = __double_as_longlong(v.y);
    const int xl = __builtin_amdgcn_readlane((int)bx, src);
    const int xh = __builtin_amdgcn_readlane((int)(bx >> 32), src);
    const int yl = __builtin_amdgcn_readlane((int)by, src);
    const int yh = __builtin_amdgcn_readlane((int)(by >> 32), src);
    return make_double2(__longlong_as_double((long long)(unsigned)xl | ((long long)xh << 32)),
                        __longlong_as_double((long long)(unsigned)yl | ((long long)yh << 32)));
}

// The smoothing, one strip of TW output columns and a run of its rows at a
// time.  Window sums are linear, so each row step scans one row of
// differences d(c) = raw(q_in, c) - raw(q_out, c) between the row entering
// the box and the row leaving it (raw(q_in) alone while the box fills), and
// the column sums take the window sums of d.  Thread t scans the 4
// consecutive widened columns e = 4t .. 4t+3 and keeps the column sums of
// the output columns j = t + NT k, whose window e = j .. j+M3-1 is the
// difference of two prefix sums read from LDS.  Rows go RPS at a time:
// their scans share one pair of barriers.
constexpr int BOX_CPT = 4;

// acc + a * b and acc - a * b for complex doubles, as fused multiply-adds
__device__ inline double2 cfma(double2 a, double2 b, double2 acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

__device__ inline double2 cfms(double2 a, double2 b, double2 acc)
{
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}

// One run: output rows [ra, rb) of the strip starting at column c0.
template <int MODE, int NT, int RPS>
__device__ __forceinline__ void box_run(const double2 *__restrict__ F,
                                        const double2 *__restrict__ S, const DbsGeom &g,
                                        double2 *__restrict__ out, int c0, int ra, int rb,
                                        double2 (*lrow)[BOX_CPT * (NT + 4)],
                                        double2 (*wtot)[NT / 64])
{
    constexpr int CPT = BOX_CPT;
    constexpr int NW = NT / 64;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int H = g.H, P = g.P, M3 = g.M3, TW = g.TW;
    const int T = (rb - ra) + M3 - 1;         // rows entering the box
    const int qa = ra - g.lo;                 // first of them
    const int e0 = t * CPT;                   // first owned widened (and output) column
    const int64_t cb = (int64_t)c0 - g.lo + e0;
    // LDS position of widened column e: four segments (e mod 4) of NT + 4
    // entries; the writes of one m by consecutive lanes are consecutive, and
    // a read of 16 consecutive columns touches 16 distinct bank groups
    auto sw = [](int e) { return (e & 3) * (NT + 4) + (e >> 2); };

    double2 v[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        v[k] = make_double2(0.0, 0.0);
    int r = ra;                               // next output row and its offset
    int64_t ro = pd_row_off(ra, H);

    // d -> global inclusive prefix sums in d, with the exclusive prefix at
    // the thread's first column in ex.  Phase 1 (before the barrier):
    // in-thread and in-wave scans; phase 2: the earlier waves, published.
    auto scan1 = [&](double2 (&d)[CPT], double2 *tot, double2 &ex) {
#pragma unroll
        for (int m = 1; m < CPT; ++m)
            d[m] = cadd(d[m], d[m - 1]);
        const double2 inc = wave_scan_incl(d[CPT - 1]);
        ex = csub(inc, d[CPT - 1]);
        if (lane == 63)
            tot[wave] = inc;
    };
    auto scan2 = [&](double2 (&d)[CPT], const double2 *tot, double2 &ex, double2 *row) {
        ex = cadd(ex, waves_before<NW>(tot, lane, wave));
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            d[m] = cadd(ex, d[m]);
            row[sw(e0 + m)] = d[m];
        }
    };
    // v += window sums of d; then the output row if the box is full.
    // Output column j = t + NT k, so each store instruction covers
    // consecutive columns; both prefix sums of its window come from LDS.
    auto update = [&](const double2 *row, int st) {
        const bool emit = st >= M3 - 1 && st < T;
        const int L = min(r, H - r);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int j = t + NT * k;
            if (j < TW) {
                const double2 top = row[sw(j + M3 - 1)];
                const double2 bot = j > 0 ? row[sw(j - 1)] : make_double2(0.0, 0.0);
                v[k] = cadd(v[k], csub(top, bot));
                if (emit && c0 + j <= L)
                    out[ro + c0 + j] = cscale(v[k], g.norm);
            }
        }
        if (emit) {
            ro += L + 1;
            ++r;
        }
    };
    // While the box fills, nothing is emitted and the rows only enter, so
    // the first P0 rows are summed per widened column without scans, in v
    // (zero and unused until then; v[m] holds column e0 + m meanwhile); at
    // the first later step one scan of those sums puts their window sums
    // into v, which is what the per-row scans would have added (window sums
    // are linear; only the order of the FP64 additions differs).
    const int P0 = ((M3 - 1) / RPS) * RPS;
    bool primed = P0 == 0;
    // Row steps st .. st + RPS - 1 from their difference rows.
    auto stepn = [&](double2 (&d)[RPS][CPT], int st) {
        if (st + RPS <= P0) {
#pragma unroll
            for (int k = 0; k < RPS; ++k)
#pragma unroll
                for (int m = 0; m < CPT; ++m)
                    v[m] = cadd(v[m], d[k][m]);
            return;
        }
        if (!primed) {
            double2 Vp[CPT], xp;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                Vp[m] = v[m];
                v[m] = make_double2(0.0, 0.0);
            }
            scan1(Vp, wtot[0], xp);
            lds_barrier();
            scan2(Vp, wtot[0], xp, lrow[0]);
            lds_barrier();
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int j = t + NT * k;
                if (j < TW) {
                    const double2 top = lrow[0][sw(j + M3 - 1)];
                    const double2 bot = j > 0 ? lrow[0][sw(j - 1)] : make_double2(0.0, 0.0);
                    v[k] = cadd(v[k], csub(top, bot));
                }
            }
            primed = true;
        }
        double2 x[RPS];
#pragma unroll
        for (int k = 0; k < RPS; ++k)
            scan1(d[k], wtot[k], x[k]);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < RPS; ++k)
            scan2(d[k], wtot[k], x[k], lrow[k]);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < RPS; ++k)
            update(lrow[k], st + k);
    };

    if constexpr (MODE == 0) {
        // K = 1: raw(q, c) = F(c) [F(q) conj F(q + c)].  conj F(q + cb + m)
        // for the CPT rows of the current block comes from two register
        // halves C (this block) and N (the next); once the block's products
        // are formed C is reloaded for the block after next, so the loads
        // are issued a whole block before their use.  Entering rows use
        // Ci/Ni, leaving rows Co/No.
        double2 Fc[CPT], Ai[CPT], Bi[CPT], Ao[CPT], Bo[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            Fc[m] = F[wrap_p(cb + m, P)];
            Ai[m] = cconj(F[wrap_p((int64_t)qa + cb + m, P)]);
            Bi[m] = cconj(F[wrap_p((int64_t)qa + CPT + cb + m, P)]);
            Ao[m] = cconj(F[wrap_p((int64_t)qa - M3 + cb + m, P)]);
            Bo[m] = cconj(F[wrap_p((int64_t)qa - M3 + CPT + cb + m, P)]);
        }
        int ldi = wrap_p((int64_t)qa + 2 * CPT + cb, P);
        int ldo = wrap_p((int64_t)qa - M3 + 2 * CPT + cb, P);
        // Row factors F(q) of the entering and leaving rows: lane k of every
        // wave loads the one of row k of the block after next (a vector load,
        // so the LDS barriers never wait for it) and each step reads its
        // row's value out of that lane.
        const int kq = lane & (2 * CPT - 1);
        int ai = wrap_p((int64_t)qa + kq, P), ao = wrap_p((int64_t)qa - M3 + kq, P);
        double2 fav = F[ai], fbv = F[ao];
        auto adv = [&](int &i) { i += 2 * CPT; if (i >= P) i -= P; if (i >= P) i %= P; };
        auto lane_c = [](double2 v, int k) {
            const long long bx = __double_as_longlong(v.x), by = __double_as_longlong(v.y);
            const int xl = __builtin_amdgcn_readlane((int)bx, k);
            const int xh = __builtin_amdgcn_readlane((int)(bx >> 32), k);
            const int yl = __builtin_amdgcn_readlane((int)by, k);
            const int yh = __builtin_amdgcn_readlane((int)(by >> 32), k);
            return make_double2(
                __longlong_as_double((long long)(unsigned)xl | ((long long)xh << 32)),
                __longlong_as_double((long long)(unsigned)yl | ((long long)yh << 32)));
        };
        double2 fa_cur = fav, fb_cur = fbv;
        auto block = [&](double2 (&Ci)[CPT], double2 (&Ni)[CPT], double2 (&Co)[CPT],
                         double2 (&No)[CPT], int sb) {
            // fa_cur / fb_cur hold rows sb .. sb + 2 CPT - 1 (lane k: row sb + k);
            // the next pair of blocks' factors are loaded at its first block
            const int kb = sb & (2 * CPT - 1);
            if (kb == 0) {
                fa_cur = fav;
                fb_cur = fbv;
                adv(ai);
                adv(ao);
                fav = F[ai];
                fbv = F[ao];
            }
            const double2 zero = make_double2(0.0, 0.0);
#pragma unroll
            for (int u0 = 0; u0 < CPT; u0 += RPS) {
                double2 d[RPS][CPT];
#pragma unroll
                for (int k = 0; k < RPS; ++k) {
                    const int u = u0 + k, st = sb + u;
                    // the leaving rows' factors are 0 while the box fills
                    const double2 a = lane_c(fa_cur, kb + u);
                    const double2 fb = lane_c(fb_cur, kb + u);
                    const double2 b = st >= M3 ? fb : zero;
#pragma unroll
                    for (int m = 0; m < CPT; ++m) {
                        const double2 ci = m + u < CPT ? Ci[m + u] : Ni[m + u - CPT];
                        const double2 co = m + u < CPT ? Co[m + u] : No[m + u - CPT];
                        d[k][m] = cmul(Fc[m], cfms(b, co, cmul(a, ci)));
                    }
                }
                if (u0 + RPS == CPT) {
                    // every value of Ci / Co has served: reload them for the
                    // block after next
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        Ci[k] = cconj(F[ldi]);
                        Co[k] = cconj(F[ldo]);
                        ldi = inc_wrap(ldi, P);
                        ldo = inc_wrap(ldo, P);
                    }
                }
                stepn(d, sb + u0);
            }
        };
        for (int sb = 0; sb < T; sb += 2 * CPT) {
            block(Ai, Bi, Ao, Bo, sb);
            if (sb + CPT < T)
                block(Bi, Ai, Bo, Ao, sb + CPT);
        }
    } else {
        // K >= 2: raw is the part sums, read one step ahead; d = entering
        // row - leaving row.  Rows past the last entering one are not read
        // (nothing is emitted from them).
        const double2 *Sb = S + cb + g.lo;     // column of element 0 in the rectangle
        auto load_d = [&](double2 (&d)[CPT], int stn) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                d[m] = make_double2(0.0, 0.0);
            if (stn < T) {
                const double2 *rin = Sb + ((int64_t)qa + stn + g.lo) * g.SC;
#pragma unroll
                for (int m = 0; m < CPT; ++m)
                    d[m] = rin[m];
                if (stn >= M3) {
                    const double2 *rout = Sb + ((int64_t)qa + stn - M3 + g.lo) * g.SC;
#pragma unroll
                    for (int m = 0; m < CPT; ++m)
                        d[m] = csub(d[m], rout[m]);
                }
            }
        };
        double2 n[RPS][CPT];
#pragma unroll
        for (int k = 0; k < RPS; ++k)
            load_d(n[k], k);
        for (int st = 0; st < T; st += RPS) {
            double2 d[RPS][CPT];
#pragma unroll
            for (int k = 0; k < RPS; ++k)
#pragma unroll
                for (int m = 0; m < CPT; ++m)
                    d[k][m] = n[k][m];
#pragma unroll
            for (int k = 0; k < RPS; ++k)
                load_d(n[k], st + RPS + k);
            stepn(d, st);
        }
    }
}

// The strips' rows laid end to end are cut into runs of g.R rows, one per
// workgroup; a run that reaches the end of a strip continues at the start
// of the next.  Strip s starts at row offset s (H + 1) - TW s (s - 1).
// Rows per step: 4 (2 for the widest strips, whose registers would not hold 4).
template <int MODE, int NT>
__global__ void __launch_bounds__(NT)
k_dbs_box(const double2 *__restrict__ F, const double2 *__restrict__ S, DbsGeom g,
          double2 *__restrict__ out)
{
    constexpr int RPS = NT >= 512 ? 2 : 4;
    __shared__ double2 lrow[RPS][BOX_CPT * (NT + 4)];   // prefix sums of the rows of a step
    __shared__ double2 wtot[RPS][NT / 64];
    auto first_row = [&](int64_t s) { return s * (g.H + 1) - (int64_t)g.TW * s * (s - 1); };
    int64_t a = (int64_t)blockIdx.x * g.R;
    const int64_t b = min(a + (int64_t)g.R, g.rows);
    while (a < b) {
        int s0 = 0, s1 = g.NS - 1;
        while (s0 < s1) {
            const int mid = (s0 + s1 + 1) >> 1;
            if (first_row(mid) <= a)
                s0 = mid;
            else
                s1 = mid - 1;
        }
        const int64_t o = first_row(s0);
        const int c0 = s0 * g.TW;
        const int ra = c0 + (int)(a - o);
        const int rb = (int)min((int64_t)c0 + (b - o), (int64_t)g.H - c0 + 1);
        box_run<MODE, NT, RPS>(F, S, g, out, c0, ra, rb, lrow, wtot);
        a += rb - ra;
    }
}

template <int MODE>
hipError_t launch_box(const DbsPlan &p, const double2 *F, const double2 *S, double2 *out,
                      hipStream_t s)
{
    const DbsGeom &g = p.g;
    const dim3 grid((unsigned)g.NSEG);
    switch (g.W) {
    case 512:  k_dbs_box<MODE, 128><<<grid, 128, 0, s>>>(F, S, g, out); break;
    case 1024: k_dbs_box<MODE, 256><<<grid, 256, 0, s>>>(F, S, g, out); break;
    default:   k_dbs_box<MODE, 512><<<grid, 512, 0, s>>>(F, S, g, out); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_parts(const T *x, uint32_t flags, const DbsPlan &p, char *ws, hipStream_t s)
{
    const int P = p.g.P;
    const int bpp = (P + MEAN_SPAN - 1) / MEAN_SPAN;
    double *psum = (double *)(ws + p.off_mean);
    double2 *F = (double2 *)(ws + p.off_F);
    const int center = (flags & HOS_NO_CENTER) ? 0 : 1;
    if (center)
        k_dbs_psum<T><<<(unsigned)(p.K * bpp), 256, 0, s>>>(x, P, bpp, psum);
    double2 *twP = (double2 *)(ws + p.off_tw);
    hipError_t e = launch_twiddles(twP, P, s);
    if (e != hipSuccess)
        return e;
    if (p.P2 == 1) {
        const FftRadices fr = factor(P);
        int CB = FFT_LDS_ELEMS / P;
        if (CB > 32)
            CB = 32;
        k_dbs_fft1<T><<<(unsigned)((p.K + CB - 1) / CB), FFT_THREADS, 0, s>>>(
            x, psum, bpp, p.K, fr, CB, twP, center, F);
    } else {
        double2 *tw1 = (double2 *)(ws + p.off_tw1), *tw2 = (double2 *)(ws + p.off_tw2);
        double2 *Tb = (double2 *)(ws + p.off_T);
        e = launch_twiddles(tw1, p.P1, s);
        if (e == hipSuccess)
            e = launch_twiddles(tw2, p.P2, s);
        if (e != hipSuccess)
            return e;
        const FftRadices f1 = factor(p.P1), f2 = factor(p.P2);
        int CB1 = FFT_LDS_ELEMS / p.P1, CB2 = FFT_LDS_ELEMS / p.P2;
        if (CB1 > 32)
            CB1 = 32;
        if (CB2 > 32)
            CB2 = 32;
        const int64_t ns1 = p.K * p.P2, ns2 = p.K * p.P1;
        k_dbs_fft_a<T><<<(unsigned)((ns1 + CB1 - 1) / CB1), FFT_THREADS, 0, s>>>(
            x, psum, bpp, p.K, p.P2, f1, CB1, tw1, twP, center, Tb);
        k_dbs_fft_b<<<(unsigned)((ns2 + CB2 - 1) / CB2), FFT_THREADS, 0, s>>>(
            Tb, p.K, p.P1, f2, CB2, tw2, F);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dbs(const void *x, int dtype, uint32_t flags, const DbsPlan &p, double *B_pd,
                      char *ws, hipStream_t s, hipEvent_t *ev)
{
    auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], s) : hipSuccess; };
    hipError_t e = mark(0);
    if (e == hipSuccess)
        e = dtype == HOS_F64 ? launch_parts((const double *)x, flags, p, ws, s)
                             : launch_parts((const float *)x, flags, p, ws, s);
    if (e == hipSuccess)
        e = mark(1);
    const double2 *F = (const double2 *)(ws + p.off_F);
    double2 *S = p.mode == 1 ? (double2 *)(ws + p.off_S) : nullptr;
    if (e == hipSuccess && p.mode == 1) {
        const dim3 grid((unsigned)((p.g.SC + 63) / 64), (unsigned)((p.SR + 63) / 64),
                        (unsigned)p.G);
        k_dbs_rawsum<<<grid, 256, 0, s>>>(F, p.g.P, p.K, p.Kg, p.g.lo, p.SR, p.g.SC, S);
        const int64_t count = (int64_t)p.SR * p.g.SC;
        if (p.G > 1)
            k_dbs_sreduce<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(S, p.G, count);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = mark(2);
    if (e == hipSuccess)
        e = p.mode == 0 ? launch_box<0>(p, F, S, (double2 *)B_pd, s)
                        : launch_box<1>(p, F, S, (double2 *)B_pd, s);
    if (e == hipSuccess)
        e = mark(3);
    return e;
}

}  // namespace hos
