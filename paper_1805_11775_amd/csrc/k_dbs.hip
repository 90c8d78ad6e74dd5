// k_dbs.hip -- the direct bispectrum method (Algorithm DBS) with the
// window-sum smoothing of Section 3 (Algorithm WS and its 2-D form).
//
// Steps 1-3: the series is cut into K parts of P samples (trailing samples
// unused), each part loses its own FP64 mean and gets a P-point DFT F_i.
// Step 4's raw bispectrum F_i(k1) F_i(k2) conj F_i(k1 + k2) / P, step 5's
// M3 x M3 box average and step 6's average over parts are all linear, so
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

// Step 2: partial sums of each part, MEAN_SPAN samples per workgroup.
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

// Step 3, P <= DBS_LDS_FFT: CB whole parts per workgroup in LDS.
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

// Step 3, P = P1 * P2 > DBS_LDS_FFT, first pass: with u = P2 n1 + n2 and
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

// The smoothing: one strip (blockIdx.y) and one run of output rows
// (blockIdx.x) per workgroup.  Thread t owns the CPT consecutive widened
// columns e = t CPT + m (for the scan) and the output columns j = t + NT k.
template <int MODE, int NT, int CPT>
__global__ void __launch_bounds__(NT)
k_dbs_box(const double2 *__restrict__ F, const double2 *__restrict__ S, DbsGeom g,
          double2 *__restrict__ out)
{
    constexpr int W = NT * CPT;
    constexpr int NW = NT / 64;
    constexpr int PADW = W + (CPT > 1 ? W / CPT : 0);
    __shared__ double2 lin[PADW], lout[PADW];
    __shared__ double2 wtot[2][NW];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int H = g.H, P = g.P, M3 = g.M3, TW = g.TW;
    const int c0 = blockIdx.y * TW;
    const int ra = c0 + blockIdx.x * g.R;
    const int rend = H - c0 + 1;              // the strip's rows are [c0, H - c0]
    if (ra >= rend)
        return;                               // whole workgroup
    const int rb = min(ra + g.R, rend);
    const int T = (rb - ra) + M3 - 1;         // rows entering the box
    const int qa = ra - g.lo;                 // first of them
    const int e0 = t * CPT;                   // first owned widened column
    const int64_t cb = (int64_t)c0 - g.lo + e0;
    auto pad = [](int e) { return CPT > 1 ? e + e / CPT : e; };

    double2 v[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        v[k] = make_double2(0.0, 0.0);

    // One row step: u (the products of the entering row, and of the leaving
    // row when has_out) -> window sums along k2 -> the column sums v; then
    // the output row when the box is full.
    // inclusive scan of the products within the wave: u[m] becomes the
    // sum up to element m of the thread's wave; returns the wave total in
    // lane 63's copy
    auto wave_scan = [&](double2 (&u)[CPT]) {
#pragma unroll
        for (int m = 1; m < CPT; ++m)
            u[m] = cadd(u[m], u[m - 1]);
        double2 tot = u[CPT - 1];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double2 y = shfl_up2(tot, d);
            if (lane >= d)
                tot = cadd(tot, y);
        }
        double2 ex = shfl_up2(tot, 1);
        if (lane == 0)
            ex = make_double2(0.0, 0.0);
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            u[m] = cadd(ex, u[m]);
        return tot;
    };
    // sum of the totals of the waves before this one
    auto wave_off = [&](const double2 *tot) {
        double2 o = make_double2(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NW - 1; ++w)
            if (w < wave)
                o = cadd(o, tot[w]);
        return o;
    };
    // sum of the first m products of a row (prefix sums stored from index 1)
    auto pfx = [&](const double2 *row, int m) {
        return m == 0 ? make_double2(0.0, 0.0) : row[pad(m - 1)];
    };

    // One row step: ui (the products of the entering row) and, when has_out,
    // uo (of the row leaving the box) -> window sums along k2 -> the column
    // sums v; then the output row once the box is full.  Two barriers: the
    // wave totals, then the complete prefix sums.
    auto step = [&](double2 (&ui)[CPT], double2 (&uo)[CPT], int st, bool has_out,
                    double2 ain, double2 aout) {
        const double2 ti = wave_scan(ui);
        if (lane == 63)
            wtot[0][wave] = ti;
        if (has_out) {
            const double2 to = wave_scan(uo);
            if (lane == 63)
                wtot[1][wave] = to;
        }
        __syncthreads();
        const double2 oi = wave_off(wtot[0]);
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            lin[pad(e0 + m)] = cadd(oi, ui[m]);
        if (has_out) {
            const double2 oo = wave_off(wtot[1]);
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                lout[pad(e0 + m)] = cadd(oo, uo[m]);
        }
        __syncthreads();
        const int r = qa + st - g.hi;         // output row when the box is full
        const bool emit = st >= M3 - 1 && st < T;
        const int L = min(r, H - r);
        const int64_t ro = emit ? pd_row_off(r, H) : 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int j = t + NT * k;
            if (j < TW) {
                const double2 hin = csub(pfx(lin, j + M3), pfx(lin, j));
                double2 acc = cadd(v[k], cmul(ain, hin));
                if (has_out) {
                    const double2 hout = csub(pfx(lout, j + M3), pfx(lout, j));
                    acc = csub(acc, cmul(aout, hout));
                }
                v[k] = acc;
                if (emit && c0 + j <= L)
                    out[ro + c0 + j] = cscale(acc, g.norm);
            }
        }
    };

    if constexpr (MODE == 0) {
        // K = 1: u_e = F(c_e) conj F(q + c_e); F(q) multiplies the row's
        // window sums.  conj F(q + cb + m) for the rows of the current
        // block of CPT steps comes from two register halves A (this block)
        // and B (the next): a value is dead once its row has passed and is
        // reloaded at once for the block after next, so each step loads one
        // value per half pair.
        double2 Fc[CPT], Ai[CPT], Bi[CPT], Ao[CPT], Bo[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            Fc[m] = F[wrap_p(cb + m, P)];
            Ai[m] = cconj(F[wrap_p((int64_t)qa + cb + m, P)]);
            Bi[m] = cconj(F[wrap_p((int64_t)qa + CPT + cb + m, P)]);
            Ao[m] = cconj(F[wrap_p((int64_t)qa - M3 + cb + m, P)]);
            Bo[m] = cconj(F[wrap_p((int64_t)qa - M3 + CPT + cb + m, P)]);
        }
        auto block = [&](double2 (&Ci)[CPT], double2 (&Ni)[CPT], double2 (&Co)[CPT],
                         double2 (&No)[CPT], int sb) {
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int st = sb + u;
                const int64_t qi = (int64_t)qa + st, qo = qi - M3;
                const double2 ain = F[wrap_p(qi, P)];
                const bool has_out = st >= M3;
                const double2 aout = has_out ? F[wrap_p(qo, P)] : make_double2(0.0, 0.0);
                double2 ui[CPT], uo[CPT];
#pragma unroll
                for (int m = 0; m < CPT; ++m) {
                    ui[m] = cmul(Fc[m], m + u < CPT ? Ci[m + u] : Ni[m + u - CPT]);
                    uo[m] = has_out ? cmul(Fc[m], m + u < CPT ? Co[m + u] : No[m + u - CPT])
                                    : make_double2(0.0, 0.0);
                }
                // Ci[u] now serves no later row: reload it for block sb + 2 CPT
                Ci[u] = cconj(F[wrap_p(qi + 2 * CPT + cb, P)]);
                Co[u] = cconj(F[wrap_p(qo + 2 * CPT + cb, P)]);
                step(ui, uo, st, has_out, ain, aout);
            }
        };
        for (int sb = 0; sb < T; sb += 2 * CPT) {
            block(Ai, Bi, Ao, Bo, sb);
            if (sb + CPT < T)
                block(Bi, Ai, Bo, Ao, sb + CPT);
        }
    } else {
        // K >= 2: the products are the part sums, read row by row.
        const double2 *Sb = S + cb + g.lo;     // column of element 0 in the rectangle
        auto load_row = [&](double2 (&u)[CPT], int64_t q) {
            const double2 *row = Sb + (q + g.lo) * g.SC;
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                u[m] = row[m];
        };
        double2 ni[CPT], no[CPT];
        load_row(ni, qa);
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            no[m] = make_double2(0.0, 0.0);
        const double2 one = make_double2(1.0, 0.0);
        for (int st = 0; st < T; ++st) {
            double2 ui[CPT], uo[CPT];
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                ui[m] = ni[m];
                uo[m] = no[m];
            }
            if (st + 1 < T)
                load_row(ni, (int64_t)qa + st + 1);
            if (st + 1 >= M3 && st + 1 < T)
                load_row(no, (int64_t)qa + st + 1 - M3);
            step(ui, uo, st, st >= M3, one, one);
        }
    }
}

template <int MODE>
hipError_t launch_box(const DbsPlan &p, const double2 *F, const double2 *S, double2 *out,
                      hipStream_t s)
{
    const DbsGeom &g = p.g;
    const dim3 grid((unsigned)g.NSEG, (unsigned)g.NS);
    switch (g.W) {
    case 256:  k_dbs_box<MODE, 256, 1><<<grid, 256, 0, s>>>(F, S, g, out); break;
    case 512:  k_dbs_box<MODE, 256, 2><<<grid, 256, 0, s>>>(F, S, g, out); break;
    case 1024: k_dbs_box<MODE, 256, 4><<<grid, 256, 0, s>>>(F, S, g, out); break;
    default:   k_dbs_box<MODE, 512, 4><<<grid, 512, 0, s>>>(F, S, g, out); break;
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
