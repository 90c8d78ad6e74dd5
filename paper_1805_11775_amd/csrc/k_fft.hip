// k_fft.hip -- FP64 complex DFTs of the windowed cumulants.
//
// The spectrum is the Fourier transform of the cumulant (Section 1), taken
// as an unnormalised DFT with the sign of Algorithm DBS's part DFT,
//     X(k) = sum_u x(u) exp(-2 pi i u k / N).
// Multi-dimensional transforms are done one axis at a time in place.  Each
// workgroup loads CB whole sequences into LDS, runs a self-sorting
// (Stockham) mixed-radix 4/2/3/5 FFT there -- every stage reads its R
// inputs per butterfly into registers, barriers, and writes them back in
// sorted position -- and stores the sequences back.  Twiddles come from a
// table of the N roots of unity built once per call with sincospi in FP64.
#include "hos_internal.h"
#include "hos_device.h"
#include "hos_fft.h"

namespace hos {

namespace {

__global__ void k_twiddle(double2 *__restrict__ tw, int N)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N)
        return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)N, &s, &c);
    tw[k] = make_double2(c, s);
}

// Sequence s starts at (s / b_in) * s_out + (s % b_in) * s_in; element k
// of it sits k * es further.  CB sequences per workgroup, each sequence's
// start computed once.  PP: two LDS buffers of CB * N complex values (sized
// at launch); each Stockham stage reads one and writes the other, so a
// thread holds one butterfly at a time -- for short transforms, where the
// in-place stages would hold registers for butterflies that do not exist.
// Otherwise one buffer and the in-place stages (all their butterfly slots
// are used once CB * N fills the LDS area).
constexpr int FFT_MAX_CB = 64;
constexpr int AXIS_PAD = 3;   // padding of the in-place axis transforms' LDS area (lds_at)

template <int R, int THREADS>
__device__ inline void stockham_pingpong(const double2 *__restrict__ src,
                                         double2 *__restrict__ dst,
                                         const double2 *__restrict__ tw, int N, int Ns, int CB,
                                         int lgN, int lgNs)
{
    constexpr int LGR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : -1;
    const int nbf = N / R, total = CB * nbf, stride = N / (Ns * R);
    const bool p2 = LGR > 0 && lgN >= 0;
    for (int u = threadIdx.x; u < total; u += THREADS) {
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
        double2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double2 x = src[cb * N + j + q * nbf];
            v[q] = q == 0 ? x : cmul(x, tw_at(tw, q * k * stride));
        }
        dft_small<R>(v, tw, N);
        const int idxD = jq * Ns * R + k;
#pragma unroll
        for (int p = 0; p < R; ++p)
            dst[cb * N + idxD + p * Ns] = v[p];
    }
    __syncthreads();
}

// factor()'s radix order as a constant: radix i of N (8s, then 4s, 2s, 3s,
// 5s), 0 past the last.
__host__ __device__ constexpr int radix_at(int N, int i)
{
    const int rs[5] = {8, 4, 2, 3, 5};
    for (int k = 0; k < 5; ++k)
        while (N % rs[k] == 0) {
            if (i == 0)
                return rs[k];
            --i;
            N /= rs[k];
        }
    return 0;
}

// stockham_pingpong with N, NS and CB fixed at compile time: the same
// arithmetic, constant indices.
template <int R, int N, int NS, int CB, int THREADS>
__device__ inline void stockham_pingpong_c(const double2 *__restrict__ src,
                                           double2 *__restrict__ dst,
                                           const double2 *__restrict__ tw)
{
    constexpr int NBF = N / R, TOTAL = CB * NBF, STRIDE = N / (NS * R);
    for (int u = threadIdx.x; u < TOTAL; u += THREADS) {
        const int cb = u / NBF, j = u % NBF, jq = j / NS, k = j % NS;
        double2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double2 x = src[cb * N + j + q * NBF];
            v[q] = q == 0 ? x : cmul(x, tw_at(tw, q * k * STRIDE));
        }
        dft_small<R>(v, tw, N);
        const int idxD = cb * N + jq * NS * R + k;
#pragma unroll
        for (int p = 0; p < R; ++p)
            dst[idxD + p * NS] = v[p];
    }
    __syncthreads();
}

// The ping-pong stages of a compile-time N from stage I on; returns the
// buffer that holds the result.
template <int N, int I, int NS, int CB, int THREADS>
__device__ inline double2 *fft_pp_c(double2 *cur, double2 *nxt, const double2 *__restrict__ tw)
{
    constexpr int R = radix_at(N, I);
    if constexpr (R == 0) {
        return cur;
    } else {
        stockham_pingpong_c<R, N, NS, CB, THREADS>(cur, nxt, tw);
        return fft_pp_c<N, I + 1, NS * R, CB, THREADS>(nxt, cur, tw);
    }
}

// global loads in flight per thread while staging: the ping-pong variant
// (short transforms, many sequences per workgroup) gains from 8; the
// in-place one (long transforms, 4-element runs per row) measured slower
constexpr int AXIS_BATCH_PP = 8;

// NC: N fixed at compile time (constant stage indices), else 0; CB is then
// axis_cb(PP, NC), the host's choice for that N.
// Ping-pong workgroups take at most 16 sequences for N <= 64 (measured: the
// 48-point passes 49 -> 41 us, with six workgroups per CU instead of three),
// else at most 32 (the 96-point passes measured slower at 16).
__host__ __device__ constexpr int axis_pp_max_cb(int N)
{
    return N <= 64 ? 16 : 32;
}

__host__ __device__ constexpr int axis_cb(bool pp, int N)
{
    return pp ? (FFT_LDS_ELEMS / (2 * N) > axis_pp_max_cb(N) ? axis_pp_max_cb(N)
                                                             : FFT_LDS_ELEMS / (2 * N))
              : (FFT_LDS_ELEMS / N > 32 ? 32 : FFT_LDS_ELEMS / N);
}

template <bool PP, int THREADS, int NC = 0>
__global__ void __launch_bounds__(THREADS)
k_fft_axis(double2 *__restrict__ data, const double2 *__restrict__ tw, FftRadices fr,
           int64_t nseq, int64_t es, int64_t b_in, int64_t s_in, int64_t s_out, int CB_,
           int live)
{
    const int CB = NC ? axis_cb(PP, NC) : CB_;
    extern __shared__ double2 sm[];
    __shared__ int64_t base[FFT_MAX_CB];
    // the in-place stages use a padded area (lds_at), the ping-pong ones not
    constexpr int PAD = PP ? 0 : AXIS_PAD;
    const int N = NC ? NC : fr.n;
    // Workgroups go to the 8 XCDs round robin.  XCD x takes the x-th eighth
    // of the sequence blocks in order (of the largest multiple of 8 of them;
    // the rest keep their place), so that neighbouring blocks -- whose
    // strided rows share cache lines -- meet in one L2 instead of each
    // fetching whole lines for half their bytes.
    const unsigned G = gridDim.x, w = blockIdx.x, G8 = G & ~7u;
    const unsigned blk = w < G8 ? (w % 8) * (G8 / 8) + w / 8 : w;
    const int64_t seq0 = (int64_t)blk * CB;
    const int tot = CB * N;
    for (int cb = threadIdx.x; cb < CB; cb += THREADS) {
        const int64_t s = seq0 + cb;
        base[cb] = s < nseq ? (s / b_in) * s_out + (s % b_in) * s_in : -1;
    }
    __syncthreads();
    // Thread t moves the elements e = t, t + THREADS, ... of the CB x N
    // block; with es == 1 k runs fastest (a sequence is contiguous), else
    // cb (the sequences are neighbours).  The pair (fast, slow) advances by
    // (THREADS mod F, THREADS / F) without a division, and AXIS_BATCH loads
    // go out before their LDS stores.
    constexpr int AXIS_BATCH = PP ? AXIS_BATCH_PP : 1;
    const int F = es == 1 ? N : CB;
    const int df = THREADS % F, ds = THREADS / F;
    {
        int f = threadIdx.x % F, sl = threadIdx.x / F;
        for (int e0 = threadIdx.x; e0 < tot; e0 += AXIS_BATCH * THREADS) {
            double2 v[AXIS_BATCH];
            int at[AXIS_BATCH];
#pragma unroll
            for (int u = 0; u < AXIS_BATCH; ++u) {
                at[u] = -1;
                if (e0 + u * THREADS < tot) {
                    const int cb = es == 1 ? sl : f, k = es == 1 ? f : sl;
                    const int64_t b = base[cb];
                    if (b >= 0) {
                        v[u] = k < live ? data[b + k * es] : make_double2(0.0, 0.0);
                        at[u] = lds_at<PAD>(cb * N + k);
                    }
                }
                f += df;
                sl += ds;
                if (f >= F) {
                    f -= F;
                    ++sl;
                }
            }
#pragma unroll
            for (int u = 0; u < AXIS_BATCH; ++u)
                if (at[u] >= 0)
                    sm[at[u]] = v[u];
        }
    }
    __syncthreads();
    double2 *cur = sm, *nxt = sm + tot;
    int Ns = 1, lgNs = 0;
    const int lg = fr.lg;
    if constexpr (NC > 0 && PP)
        cur = fft_pp_c<NC, 0, 1, axis_cb(true, NC), THREADS>(sm, sm + tot, tw);
    else if constexpr (NC > 0)
        fft_lds_c<NC, 1, axis_cb(false, NC), THREADS, PAD>(sm, tw);
    for (int st = 0; NC == 0 && st < 16 && fr.r[st] > 0; ++st) {
        const int R = fr.r[st];
        if constexpr (PP) {
            if (R == 8)
                stockham_pingpong<8, THREADS>(cur, nxt, tw, N, Ns, CB, lg, lgNs);
            else if (R == 4)
                stockham_pingpong<4, THREADS>(cur, nxt, tw, N, Ns, CB, lg, lgNs);
            else if (R == 2)
                stockham_pingpong<2, THREADS>(cur, nxt, tw, N, Ns, CB, lg, lgNs);
            else if (R == 3)
                stockham_pingpong<3, THREADS>(cur, nxt, tw, N, Ns, CB, lg, lgNs);
            else
                stockham_pingpong<5, THREADS>(cur, nxt, tw, N, Ns, CB, lg, lgNs);
            double2 *t = cur;
            cur = nxt;
            nxt = t;
        } else {
            if (R == 8)
                stockham_stage<8, THREADS, FFT_LDS_ELEMS, PAD>(sm, tw, N, Ns, CB, lg, lgNs);
            else if (R == 4)
                stockham_stage<4, THREADS, FFT_LDS_ELEMS, PAD>(sm, tw, N, Ns, CB, lg, lgNs);
            else if (R == 2)
                stockham_stage<2, THREADS, FFT_LDS_ELEMS, PAD>(sm, tw, N, Ns, CB, lg, lgNs);
            else if (R == 3)
                stockham_stage<3, THREADS, FFT_LDS_ELEMS, PAD>(sm, tw, N, Ns, CB, lg, lgNs);
            else
                stockham_stage<5, THREADS, FFT_LDS_ELEMS, PAD>(sm, tw, N, Ns, CB, lg, lgNs);
        }
        Ns *= R;
        lgNs += R == 8 ? 3 : R == 4 ? 2 : R == 2 ? 1 : 0;
    }
    {
        int f = threadIdx.x % F, sl = threadIdx.x / F;
        for (int e = threadIdx.x; e < tot; e += THREADS) {
            const int cb = es == 1 ? sl : f, k = es == 1 ? f : sl;
            const int64_t b = base[cb];
            if (b >= 0)
                data[b + k * es] = cur[lds_at<PAD>(cb * N + k)];
            f += df;
            sl += ds;
            if (f >= F) {
                f -= F;
                ++sl;
            }
        }
    }
}

// Elements k >= live of every sequence are taken as 0 and not read (live =
// N: all of them).
void fft_axis(double2 *d, const double2 *tw, const FftRadices &fr, int64_t nseq, int64_t es,
              int64_t b_in, int64_t s_in, int64_t s_out, hipStream_t s, int live = -1)
{
    if (live < 0)
        live = fr.n;
    // ping-pong while both buffers of >= 8 sequences fit the 64 KB area
    // (N <= 256), else in place
    // (axis_cb: a smaller LDS area lets more workgroups share a CU, and 16
    // neighbouring sequences still make 256-byte runs of a strided axis)
    int CB = axis_cb(true, fr.n);
    if (CB >= 8) {
        const int64_t blocks = (nseq + CB - 1) / CB;
        const size_t lds = 2 * (size_t)CB * fr.n * sizeof(double2);
        // the trispectrum's and order five's default sizes at compile time
        if (fr.n == 96)
            k_fft_axis<true, FFT_THREADS, 96><<<blocks, FFT_THREADS, lds, s>>>(
                d, tw, fr, nseq, es, b_in, s_in, s_out, CB, live);
        else if (fr.n == 48)
            k_fft_axis<true, FFT_THREADS, 48><<<blocks, FFT_THREADS, lds, s>>>(
                d, tw, fr, nseq, es, b_in, s_in, s_out, CB, live);
        else
            k_fft_axis<true, FFT_THREADS><<<blocks, FFT_THREADS, lds, s>>>(
                d, tw, fr, nseq, es, b_in, s_in, s_out, CB, live);
        return;
    }
    // in place: long transforms fill the LDS area with few sequences, so a
    // workgroup of 1024 threads takes one butterfly per thread and stage
    CB = FFT_LDS_ELEMS / fr.n;
    if (CB > 32)
        CB = 32;
    const int64_t blocks = (nseq + CB - 1) / CB;
    const size_t lds = (size_t)lds_slots<AXIS_PAD>(CB * fr.n) * sizeof(double2);
    if (fr.n == 1024)
        k_fft_axis<false, 1024, 1024><<<blocks, 1024, lds, s>>>(d, tw, fr, nseq, es, b_in, s_in,
                                                               s_out, CB, live);
    else if (fr.n >= 512)
        k_fft_axis<false, 1024><<<blocks, 1024, lds, s>>>(d, tw, fr, nseq, es, b_in, s_in, s_out,
                                                         CB, live);
    else
        k_fft_axis<false, FFT_THREADS><<<blocks, FFT_THREADS, lds, s>>>(d, tw, fr, nseq, es,
                                                                       b_in, s_in, s_out, CB,
                                                                       live);
}

}  // namespace

bool fft_size_ok(int N)
{
    if (N < 2 || N > FFT_LDS_ELEMS)
        return false;
    int m = N;
    for (int r : {2, 3, 5})
        while (m % r == 0)
            m /= r;
    return m == 1;
}

hipError_t launch_twiddles(double2 *tw, int N, hipStream_t s)
{
    k_twiddle<<<(N + 255) / 256, 256, 0, s>>>(tw, N);
    return hipGetLastError();
}


}  // namespace hos

namespace hos {

// In-place 2-D DFTs of `count` contiguous N x N row-major complex grids
// whose input is nonzero only in the first `rows` rows and `cols` columns;
// nothing outside that corner is read (it may hold anything).  The columns
// k2 < cols are transformed first (their elements k1 >= rows taken as 0),
// then every row (its elements k2 >= cols taken as 0).
namespace {

// The adjoint's lag weights straight from the residual's DFT along k2: CB
// rows m1 of one series' grid (its k1 pass done; columns k2 >= live are 0)
// are transformed in LDS, and each row writes the lag table rows it holds,
// G(w1, w2) = W3(w) Re(row[w2 mod N]) for w1 = m1 and m1 - N within [-M, M],
// every w2 in [-M, M], 0 off the hexagon (N >= 2M: every lag has one grid
// point).  The N x N grid is never written.  blockIdx = (row block, series
// of the group).
template <int THREADS>
__global__ void __launch_bounds__(THREADS)
k_adj_grows(const double2 *__restrict__ grids, const SeriesDesc *__restrict__ sd,
            const int32_t *__restrict__ gser, int64_t first, const double2 *__restrict__ tw,
            FftRadices fr, int CB, int live, int window, char *__restrict__ ws)
{
    extern __shared__ double2 sm[];
    __shared__ double dwin[ADJ_MAX_M + 1];   // Parzen weights d(|m|) (1 without a window)
    const int N = fr.n;
    const SeriesDesc &d = sd[gser[first + blockIdx.y]];
    const int M = d.M, S = 2 * M + 1;
    const int m1_0 = blockIdx.x * CB;
    const int nrow = N - m1_0 < CB ? N - m1_0 : CB;
    const double2 *F = grids + (int64_t)blockIdx.y * N * N + (int64_t)m1_0 * N;
    for (int m = threadIdx.x; m <= M; m += THREADS)
        dwin[m] = window != HOS_WIN_NONE ? parzen_d(m, M) : 1.0;
    for (int e = threadIdx.x; e < CB * N; e += THREADS) {
        const int cb = e / N, k = e - cb * N;
        sm[lds_at<AXIS_PAD>(e)] = cb < nrow && k < live ? F[e] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    fft_lds<THREADS, FFT_LDS_ELEMS, AXIS_PAD>(sm, tw, fr, CB);
    double *G = (double *)(ws + d.ws_off + d.o_gtab);
    // row cb holds w1 = m1 (when m1 <= M) and w1 = m1 - N (when m1 >= N - M);
    // (cb, j) advance by (THREADS / S, THREADS mod S) without a division
    for (int alias = 0; alias < 2; ++alias) {
        int cb = threadIdx.x / S, j = threadIdx.x - cb * S;
        const int dcb = THREADS / S, dj = THREADS - dcb * S;
        for (; cb < nrow; ) {
            const int m1 = m1_0 + cb, w1 = alias ? m1 - N : m1, w2 = j - M;
            if (w1 >= -M && w1 <= M) {
                const int m2 = w2 < 0 ? w2 + N : w2, dd = w1 - w2;
                double g = 0.0;
                if (dd >= -M && dd <= M) {
                    double w = dwin[abs(w1)] * dwin[abs(w2)];
                    if (window == HOS_WIN_PARZEN)
                        w *= dwin[abs(dd)];
                    g = w * sm[lds_at<AXIS_PAD>(cb * N + m2)].x;
                }
                G[(int64_t)(w1 + M) * S + j] = g;
            }
            cb += dcb;
            j += dj;
            if (j >= S) {
                j -= S;
                ++cb;
            }
        }
    }
}

}  // namespace

hipError_t launch_adj_gweights(const FftGroup &gr, const SeriesDesc *sd, const int32_t *gser,
                               int window, char *ws, hipStream_t s)
{
    double2 *d = (double2 *)(ws + gr.grid_off);
    const double2 *tw = (const double2 *)(ws + gr.twid_off);
    const int N = gr.N;
    const FftRadices fr = factor(N);
    const int64_t N2 = (int64_t)N * N;
    // the residual sits on the principal domain: rows k1 <= H = (N - 1) / 2,
    // columns k2 <= H / 2
    const int H = (N - 1) / 2, rows = H + 1, cols = H / 2 + 1;
    fft_axis(d, tw, fr, (int64_t)gr.count * cols, N, cols, 1, N2, s, rows);   // along k1
    int CB = FFT_LDS_ELEMS / N;
    if (CB > 32)
        CB = 32;
    const dim3 grid((unsigned)((N + CB - 1) / CB), (unsigned)gr.count);
    const size_t lds = (size_t)lds_slots<AXIS_PAD>(CB * N) * sizeof(double2);
    if (N >= 512)
        k_adj_grows<1024><<<grid, 1024, lds, s>>>(d, sd, gser, gr.first, tw, fr, CB, cols, window,
                                                  ws);
    else
        k_adj_grows<FFT_THREADS><<<grid, FFT_THREADS, lds, s>>>(d, sd, gser, gr.first, tw, fr, CB,
                                                                cols, window, ws);
    return hipGetLastError();
}

}  // namespace hos

// ------------------------------------------------------------------------
// Principal-domain spectra of a batch.  Only 0 <= k2 <= k1, k1 + k2 < N/2
// is returned, so k2 <= N/4 and k1 < N/2: the 2-D DFT runs as row
// transforms (along m2) that keep the K2 = N/4 + 1 lowest k2, then column
// transforms of those K2 columns that keep the principal-domain k1.  The
// windowed, folded cumulant is formed directly in LDS by the row pass, so
// no N x N grid is written.
// ------------------------------------------------------------------------
namespace hos {

namespace {

__device__ inline int pd_len(int k1, int H) { return k1 <= H ? min(k1, H - k1) + 1 : 0; }

// First packed index of principal-domain row k1 (rows hold min(k1, H - k1)
// + 1 points: k1 + 1 up to h = floor(H / 2), H - k1 + 1 after).
__device__ inline int pd_row_start(int k1, int H)
{
    const int h = H / 2, p = k1 < h + 1 ? k1 : h + 1;
    int start = p * (p + 1) / 2;
    if (k1 > h + 1)
        start += (k1 - h - 1) * (H + 1) - ((k1 - 1) * k1 / 2 - h * (h + 1) / 2);
    return start;
}

// The windowed cumulant folded onto grid point (m1, m2) of the N x N DFT
// grid: the sum of W3 c3 over the lags w = m (mod N).  Lag w lies in
// [-M, M] and N >= 2M, so each axis has one alias candidate -- the centred
// representative m or m - N -- except at m = M when N = 2M, where both
// candidates +-M carry a Parzen factor d(M) = 0 (and N = 2M is allowed only
// with a Parzen window).  So the fold is the centred lag's term alone: one
// table read per grid point, no loop.  The square's corners |w1 - w2| > M
// count only without the Parzen product (its d(w1 - w2) vanishes there)
// and only when the table holds them (amax > M).
struct FoldArgs {
    const double *cfull;
    const double *dwin;   // d(0..M) (or 1: no window)
    double inv_norm;      // 1 / (n s^3), formed once per thread
    int M, amax, N;
    bool pdiff;           // Parzen product: d on the difference too
};

// Branch-free: a point off the support reads table entry 0 and d(0) and is
// then selected to 0, so the reads of several points can be in flight at
// once.  On the support the span a = max(0, w1, w2) - min(0, w1, w2) is at
// most amax (the hexagon has a <= M; the corners, only without the Parzen
// product, a <= 2M = amax), so the table entry is c3_table_sum's.
__device__ __attribute__((always_inline)) inline double fold_centred(const FoldArgs &f, int m1,
                                                                     int m2)
{
    const int w1 = m1 <= f.N / 2 ? m1 : m1 - f.N;
    const int w2 = m2 <= f.N / 2 ? m2 : m2 - f.N;
    const int dw = w1 - w2;
    const bool in = m1 < f.N && abs(w1) <= f.M && abs(w2) <= f.M &&
                    (abs(dw) <= f.M || (!f.pdiff && f.amax > f.M));
    const int mn = min(0, min(w1, w2)), mx = max(0, max(w1, w2));
    const int a = mx - mn, b = (w1 + w2) - mn - mx - mn;
    const int row = a <= f.M ? a : a - f.M - 1;
    const unsigned off = in ? (unsigned)(row * (f.M + 1) + b) : 0u;
    const double c = f.cfull[off];
    const double wt = f.dwin[in ? abs(w1) : 0] * f.dwin[in ? abs(w2) : 0] *
                      (f.pdiff ? f.dwin[in ? abs(dw) : 0] : 1.0);
    return in ? (wt * f.inv_norm) * c : 0.0;
}

constexpr int PD_LDS_ELEMS = 2048;   // complex doubles per workgroup (32 KB): 4+ per CU
constexpr int PD_PAD = 3;            // the batch spectra's LDS padding (lds_at)

// Sequences per workgroup of the batch spectra: PD_LDS_ELEMS complex values
// for N >= 512, PD_LDS_ELEMS / 2 below (the smaller area lets six
// workgroups share a CU instead of four; measured faster for N <= 256 and
// slower at 512), at most 32 sequences.
__host__ __device__ constexpr int pd_cb(int N)
{
    return N <= 0 ? 1
                  : (N >= 512 ? PD_LDS_ELEMS : PD_LDS_ELEMS / 2) / N > 32
                        ? 32
                        : (N >= 512 ? PD_LDS_ELEMS : PD_LDS_ELEMS / 2) / N;
}

// Workgroups are dispatched to the 8 XCDs round robin by their linear index,
// and each XCD has its own L2.  The spectra kernels read one series' table
// (rows) or grid (columns) from every one of that series' workgroups, so
// the grid is laid out to keep a series on one XCD: linear index w runs on
// XCD w % 8, and the k-th workgroup of XCD x (k = w / 8) takes block k % NBLK
// of series x + 8 (k / NBLK).  Returns false for the padding workgroups.
constexpr int N_XCD = 8;

__device__ inline bool xcd_series_block(int count, int nblk, int &series, int &blk)
{
    const int w = blockIdx.x, x = w % N_XCD, k = w / N_XCD;
    series = x + N_XCD * (k / nblk);
    blk = k % nblk;
    return series < count;
}

inline unsigned xcd_grid(int count, int nblk)
{
    return (unsigned)(N_XCD * ((count + N_XCD - 1) / N_XCD) * nblk);
}

// Rows: blockIdx.y = series of group g, blockIdx.x = block of 2 CBP rows m1.
// The folded rows are real, so rows m1 and m1 + 1 travel as the real and
// imaginary parts of one complex sequence; after its DFT Z,
//   X_{m1}(k) = (Z(k) + conj Z(N-k)) / 2,  X_{m1+1}(k) = (Z(k) - conj Z(N-k)) / 2i.
// T1[m1][k2] (k2 < K2) goes to the series' grid region.
// NC: N fixed at compile time (a power of two, >= 64; CBP is then pd_cb(NC)),
// else 0.  POW2: N is a power of two.  At least 3 waves per SIMD: the LDS
// area admits 3 workgroups per CU even at its largest.
template <bool POW2, int NC>
__global__ void __launch_bounds__(FFT_THREADS, 3)
k_pd_rows(const SeriesDesc *__restrict__ sd, const int32_t *__restrict__ gser, int first,
          int count, int nblk, char *__restrict__ ws, const double2 *__restrict__ tw,
          FftRadices fr, int CBP_, int window)
{
    const int N = NC ? NC : fr.n, CBP = NC ? pd_cb(NC) : CBP_;
    // LDS sized at launch: the padded CBP x N area, then d(m) for m = 0..N/2
    // (M <= N/2)
    extern __shared__ double2 sm[];
    double *dwin = (double *)(sm + lds_slots<PD_PAD>(CBP * N));
    int si, blk;
    if (!xcd_series_block(count, nblk, si, blk))
        return;
    const SeriesDesc &d = sd[gser[first + si]];
    const int M = d.M, K2 = N / 4 + 1, half = N / 2;
    const char *r = ws + d.ws_off;
    const bool pz = window != HOS_WIN_NONE;            // d on the lags
    const bool pdiff = window == HOS_WIN_PARZEN;        // and on their difference
    for (int m = threadIdx.x; m <= M; m += FFT_THREADS)
        dwin[m] = pz ? parzen_d(m, M) : 1.0;
    __syncthreads();
    // Batches hold the hexagon |w1|, |w2|, |w1 - w2| <= M only, so the span
    // a of a lag is at most M and its table row is a itself (c3_table_sum
    // with amax = M); table offsets stay below (M + 1)^2 and fit 32 bits.
    const double *cf = (const double *)(r + d.o_cfull);
    const double inv_norm = 1.0 / ((const double *)(r + d.o_stats))[3];
    const int m1_0 = blk * 2 * CBP;
    // A wave covers all CBP row pairs of 64 / CBP consecutive columns: off
    // the table's rows (w2 beyond w1, or of the other sign) a point reads
    // the table down a column or a diagonal, and the block's 2 CBP
    // consecutive rows then share cache lines there, where 64 consecutive
    // columns of one row would touch 64 lines.  Element e = m2 CBP + p of
    // thread t runs over e = t, t + FFT_THREADS, ...: (m2, p) advances by
    // (FFT_THREADS / CBP, FFT_THREADS % CBP) with a carry, no division.
    // The windowed, folded value of grid point (m1, m2) is the centred lag's
    // term alone (fold_centred); the products keep its order, so the values
    // equal that helper's bit for bit.  The table and d(m) reads are not
    // branched on: a point off the hexagon reads entry 0 and d(0) and its
    // value is then selected to 0, so the loads of FOLD_BATCH iterations (two
    // points each) go out together instead of one latency per point.
    constexpr int FOLD_BATCH = 4;
    {
        const int dp = FFT_THREADS % CBP, dm = FFT_THREADS / CBP;
        int p = threadIdx.x % CBP, m2 = threadIdx.x / CBP;
        for (int e0 = threadIdx.x; e0 < CBP * N; e0 += FOLD_BATCH * FFT_THREADS) {
            double c[FOLD_BATCH][2], w[FOLD_BATCH][2];
            bool in[FOLD_BATCH][2];
            int at[FOLD_BATCH];
#pragma unroll
            for (int u = 0; u < FOLD_BATCH; ++u) {
                const int w2 = m2 <= half ? m2 : m2 - N;
                const bool cin = e0 + u * FFT_THREADS < CBP * N && abs(w2) <= M;
                const double d2 = dwin[cin ? abs(w2) : 0];
                at[u] = lds_at<PD_PAD>(p * N + m2);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int m1 = m1_0 + 2 * p + h;
                    const int w1 = m1 <= half ? m1 : m1 - N, dw = w1 - w2;
                    const bool ok = cin && m1 < N && abs(w1) <= M && abs(dw) <= M;
                    const int mn = min(0, min(w1, w2)), mx = max(0, max(w1, w2));
                    const unsigned off =
                        ok ? (unsigned)((mx - mn) * (M + 1) + (w1 + w2 - mx - 2 * mn)) : 0u;
                    c[u][h] = cf[off];
                    w[u][h] = dwin[ok ? abs(w1) : 0] * d2 * (pdiff ? dwin[ok ? abs(dw) : 0] : 1.0);
                    in[u][h] = ok;
                }
                p += dp;
                m2 += dm;
                if (p >= CBP) {
                    p -= CBP;
                    ++m2;
                }
            }
#pragma unroll
            for (int u = 0; u < FOLD_BATCH; ++u)
                if (e0 + u * FFT_THREADS < CBP * N)
                    sm[at[u]] = make_double2(in[u][0] ? (w[u][0] * inv_norm) * c[u][0] : 0.0,
                                             in[u][1] ? (w[u][1] * inv_norm) * c[u][1] : 0.0);
        }
    }
    __syncthreads();
    if constexpr (NC > 0)
        fft_lds_c<NC, 1, pd_cb(NC), FFT_THREADS, PD_PAD>(sm, tw);
    else
        fft_lds<FFT_THREADS, PD_LDS_ELEMS, PD_PAD, POW2>(sm, tw, fr, CBP);
    // T1 is column-major, [k2][m1], so that the column pass reads whole
    // columns; a thread writes rows m1, m1 + 1 of one column and the CBP
    // threads of a column write its 2 CBP consecutive rows
    double2 *T1 = (double2 *)(ws + d.grid_off);
    {
        const int dp = FFT_THREADS % CBP, dk = FFT_THREADS / CBP;
        int p = threadIdx.x % CBP, k2 = threadIdx.x / CBP;
        for (int e = threadIdx.x; e < CBP * K2; e += FFT_THREADS) {
            const int m1 = m1_0 + 2 * p;
            const double2 z = sm[lds_at<PD_PAD>(p * N + k2)],
                          zc = sm[lds_at<PD_PAD>(p * N + (k2 == 0 ? 0 : N - k2))];
            // conj(Z(N-k)) = (zc.x, -zc.y)
            double2 *col = T1 + (int64_t)k2 * N;
            if (m1 < N)
                col[m1] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
            if (m1 + 1 < N)
                col[m1 + 1] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
            p += dp;
            k2 += dk;
            if (p >= CBP) {
                p -= CBP;
                ++k2;
            }
        }
    }
}

// Columns: blockIdx.x = block of CB columns k2 < K2; transforms along m1 and
// writes the principal-domain points of those columns.
template <bool POW2, int NC>
__global__ void __launch_bounds__(FFT_THREADS, 3)
k_pd_cols(const SeriesDesc *__restrict__ sd, const int32_t *__restrict__ gser, int first,
          int count, int nblk, const char *__restrict__ ws, const double2 *__restrict__ tw,
          FftRadices fr, int CB_, double2 *__restrict__ B_pd)
{
    const int N = NC ? NC : fr.n, CB = NC ? pd_cb(NC) : CB_;
    // LDS sized at launch: the padded CB x N area, then the packed starts of
    // rows k1 = 0..N/2
    extern __shared__ double2 sm[];
    int *rowstart = (int *)(sm + lds_slots<PD_PAD>(CB * N));
    int si, blk;
    if (!xcd_series_block(count, nblk, si, blk))
        return;
    const SeriesDesc &d = sd[gser[first + si]];
    const int K2 = N / 4 + 1, H = (N - 1) / 2;
    const int k2_0 = blk * CB;
    // the block's CB columns are contiguous in T1 ([k2][m1]): element e =
    // cb N + m1 of the block sits at T1 + k2_0 N + e
    const double2 *T1 = (const double2 *)(ws + d.grid_off) + (int64_t)k2_0 * N;
    const int live = (K2 - k2_0 < CB ? K2 - k2_0 : CB) * N;   // elements of columns k2 < K2
    // COL_BATCH loads in flight per thread before their LDS stores (4 where
    // the radix-3/5 stages already set the register budget); past the live
    // columns a thread reads element 0 (always live) and stores 0
    constexpr int COL_BATCH = POW2 ? 8 : 4;
    for (int e0 = threadIdx.x; e0 < CB * N; e0 += COL_BATCH * FFT_THREADS) {
        double2 v[COL_BATCH];
#pragma unroll
        for (int u = 0; u < COL_BATCH; ++u) {
            const int e = e0 + u * FFT_THREADS;
            v[u] = T1[e < live ? e : 0];
        }
#pragma unroll
        for (int u = 0; u < COL_BATCH; ++u) {
            const int e = e0 + u * FFT_THREADS;
            if (e < CB * N)
                sm[lds_at<PD_PAD>(e)] = e < live ? v[u] : make_double2(0.0, 0.0);
        }
    }
    for (int a = threadIdx.x; a <= H && a < N / 2 + 1; a += FFT_THREADS)
        rowstart[a] = pd_row_start(a, H);
    __syncthreads();
    if constexpr (NC > 0)
        fft_lds_c<NC, 1, pd_cb(NC), FFT_THREADS, PD_PAD>(sm, tw);
    else
        fft_lds<FFT_THREADS, PD_LDS_ELEMS, PD_PAD, POW2>(sm, tw, fr, CB);
    // consecutive threads take consecutive k2 of one row k1: the CB points a
    // row holds in this block are contiguous in the packed output; (cb, k1)
    // advances by (FFT_THREADS mod CB, FFT_THREADS / CB) with a carry
    const int half = H + 1;   // k1 <= H
    double2 *out = B_pd + d.pd_off;
    {
        const int dcb = FFT_THREADS % CB, dk = FFT_THREADS / CB;
        int cb = threadIdx.x % CB, k1 = threadIdx.x / CB;
        for (int e = threadIdx.x; e < CB * half; e += FFT_THREADS) {
            const int k2 = k2_0 + cb;
            if (k2 < K2 && k2 <= k1 && k1 + k2 <= H)
                out[rowstart[k1] + k2] = sm[lds_at<PD_PAD>(cb * N + k1)];
            cb += dcb;
            k1 += dk;
            if (cb >= CB) {
                cb -= CB;
                ++k1;
            }
        }
    }
}


// The full N x N spectrum of one series: fold + window into LDS, row DFTs with
// two real rows per complex sequence (as k_pd_rows), every k2 written to B;
// the column pass then runs in place (launch_fft_cols).
// NC: N fixed at compile time (1024: the FFT stages' indices and the loop
// counts become constants; CBP is then ELEMS / NC), else 0.
template <int ELEMS, int THREADS, int NC = 0>
__global__ void __launch_bounds__(THREADS)
k_full_rows(const double *__restrict__ cfull, const double *__restrict__ stats, int M,
            int amax, const double2 *__restrict__ tw, FftRadices fr, int CBP_, int window,
            double2 *__restrict__ B)
{
    __shared__ double2 sm[ELEMS];
    __shared__ double dwin[FFT_LDS_ELEMS / 2 + 1];
    const int N = NC ? NC : fr.n, CBP = NC ? ELEMS / NC : CBP_;
    const bool pz = window != HOS_WIN_NONE;            // d on the lags
    for (int m = threadIdx.x; m <= M; m += THREADS)
        dwin[m] = pz ? parzen_d(m, M) : 1.0;
    __syncthreads();
    const FoldArgs f = {cfull, dwin, 1.0 / stats[3], M, amax, N, window == HOS_WIN_PARZEN};
    const int m1_0 = blockIdx.x * 2 * CBP;
#pragma unroll 4
    for (int e = threadIdx.x; e < CBP * N; e += THREADS) {
        const int p = e / N, m2 = e - p * N, m1 = m1_0 + 2 * p;
        sm[e] = make_double2(fold_centred(f, m1, m2), fold_centred(f, m1 + 1, m2));
    }
    __syncthreads();
    if constexpr (NC > 0)
        fft_lds_c<NC, 1, ELEMS / NC, THREADS, 0>(sm, tw);
    else
        fft_lds<THREADS, ELEMS>(sm, tw, fr, CBP);
    for (int e = threadIdx.x; e < CBP * N; e += THREADS) {
        const int p = e / N, k = e - p * N, m1 = m1_0 + 2 * p;
        const double2 z = sm[p * N + k], zc = sm[p * N + (k == 0 ? 0 : N - k)];
        if (m1 < N)
            B[(int64_t)m1 * N + k] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        if (m1 + 1 < N)
            B[(int64_t)(m1 + 1) * N + k] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
}

// The trispectrum's N^3 grid: fold + six-factor window of c4 into LDS for
// lines of fixed (m1, m2) (line L = m1 N + m2), transforms along m3 with two
// real lines per complex sequence, every k3 written to T; the k2 and k1
// passes follow (launch_fft3_tail).
__global__ void __launch_bounds__(FFT_THREADS)
k_tri_lines(const double *__restrict__ c4, int M, const double2 *__restrict__ tw, FftRadices fr,
            int CBP, int window, double2 *__restrict__ T)
{
    __shared__ double2 sm[PD_LDS_ELEMS];
    __shared__ double dwin[PD_LDS_ELEMS / 2 + 1];
    const int N = fr.n;
    const int64_t lines = (int64_t)N * N;
    const int side = 2 * M + 1;
    const bool pz = window != HOS_WIN_NONE;            // d on the lags
    const bool pdiff = window == HOS_WIN_PARZEN;        // and on their differences
    for (int m = threadIdx.x; m <= M; m += FFT_THREADS)
        dwin[m] = pz ? parzen_d(m, M) : 1.0;
    __syncthreads();
    // The fold onto grid point (m1, m2, m3) is the centred lag's term alone:
    // N >= 2M, so an axis has one alias candidate in [-M, M] -- or, at m = M
    // when N = 2M, two (+-M) whose Parzen factor d(M) is 0, as is the
    // centred one's (the trispectrum's spectrum takes the Parzen window
    // only).  Branch-free: a point off the support reads the cube's entry 0
    // and d(0) and is then selected to 0, so the reads of several points are
    // in flight at once.  The window's products keep the alias sum's order.
    auto fold = [&](int64_t L, int m3) {
        const int m1 = (int)(L / N), m2 = (int)(L - (int64_t)m1 * N);
        const int t1 = m1 <= N / 2 ? m1 : m1 - N, t2 = m2 <= N / 2 ? m2 : m2 - N,
                  t3 = m3 <= N / 2 ? m3 : m3 - N;
        const bool ok = L < lines && abs(t1) <= M && abs(t2) <= M && abs(t3) <= M &&
                        abs(t2 - t1) <= M && abs(t3 - t1) <= M && abs(t3 - t2) <= M;
        const int64_t at =
            ok ? ((int64_t)(t1 + M) * side + (t2 + M)) * side + (t3 + M) : 0;
        const double c = c4[at];
        const int a1 = ok ? abs(t1) : 0, a2 = ok ? abs(t2) : 0, a3 = ok ? abs(t3) : 0;
        const double wl = dwin[a1] * dwin[a2] * dwin[a3];
        const double w = pdiff ? wl * dwin[ok ? abs(t2 - t1) : 0] * dwin[ok ? abs(t3 - t1) : 0] *
                                     dwin[ok ? abs(t3 - t2) : 0]
                               : wl;
        return ok ? 0.0 + w * c : 0.0;
    };
    const int64_t L0 = (int64_t)blockIdx.x * 2 * CBP;
#pragma unroll 4
    for (int e = threadIdx.x; e < CBP * N; e += FFT_THREADS) {
        const int p = e / N, m3 = e - p * N;
        sm[e] = make_double2(fold(L0 + 2 * p, m3), fold(L0 + 2 * p + 1, m3));
    }
    __syncthreads();
    fft_lds<FFT_THREADS, PD_LDS_ELEMS>(sm, tw, fr, CBP);
    for (int e = threadIdx.x; e < CBP * N; e += FFT_THREADS) {
        const int p = e / N, k = e - p * N;
        const int64_t L = L0 + 2 * p;
        const double2 z = sm[p * N + k], zc = sm[p * N + (k == 0 ? 0 : N - k)];
        if (L < lines)
            T[L * N + k] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        if (L + 1 < lines)
            T[(L + 1) * N + k] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
}

}  // namespace

hipError_t launch_pd_spectra(const BatchHeader &h, const char *dplan, int window, char *ws,
                             double *B_pd, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    const int32_t *gser = (const int32_t *)(dplan + h.gseries_off);
    const FftGroup *groups = (const FftGroup *)((const char *)&h + h.groups_off);
    for (int g = 0; g < (int)h.n_groups; ++g) {
        const FftGroup &gr = groups[g];
        const int N = gr.N;
        double2 *tw = (double2 *)(ws + gr.twid_off);
        hipError_t e = launch_twiddles(tw, N, s);
        if (e != hipSuccess)
            return e;
        const FftRadices fr = factor(N);
        const int CB = pd_cb(N);
        const int K2 = N / 4 + 1;
        if (CB >= 1) {
            const int rb = (N + 2 * CB - 1) / (2 * CB), cbk = (K2 + CB - 1) / CB;
            const size_t area = (size_t)lds_slots<PD_PAD>(CB * N) * sizeof(double2);
            const size_t lds_r = area + (size_t)(N / 2 + 1) * sizeof(double),
                         lds_c = area + (size_t)(N / 2 + 1) * sizeof(int);
            const dim3 gr_r(xcd_grid(gr.count, rb)), gr_c(xcd_grid(gr.count, cbk));
            const int first = (int)gr.first;
            double2 *Bp = (double2 *)B_pd;
#define HOS_PD_LAUNCH(P2, NCV)                                                              \
    do {                                                                                    \
        k_pd_rows<P2, NCV><<<gr_r, FFT_THREADS, lds_r, s>>>(sd, gser, first, gr.count, rb, \
                                                            ws, tw, fr, CB, window);        \
        k_pd_cols<P2, NCV><<<gr_c, FFT_THREADS, lds_c, s>>>(sd, gser, first, gr.count, cbk, \
                                                            ws, tw, fr, CB, Bp);            \
    } while (0)
            switch (N) {
            case 64: HOS_PD_LAUNCH(true, 64); break;
            case 128: HOS_PD_LAUNCH(true, 128); break;
            case 256: HOS_PD_LAUNCH(true, 256); break;
            case 512: HOS_PD_LAUNCH(true, 512); break;
            case 1024: HOS_PD_LAUNCH(true, 1024); break;
            case 2048: HOS_PD_LAUNCH(true, 2048); break;
            default:
                if (fr.lg >= 0)
                    HOS_PD_LAUNCH(true, 0);
                else
                    HOS_PD_LAUNCH(false, 0);
            }
#undef HOS_PD_LAUNCH
        } else {
            return hipErrorInvalidValue;   // N > 2048: not planned for batches
        }
    }
    return hipGetLastError();
}

// Fold, window and row transforms of one series' N x N spectrum into B.
hipError_t launch_full_rows(const double *cfull, const double *stats, int M, int amax, int N,
                            int window, const double2 *tw, double *B, hipStream_t s)
{
    const FftRadices fr = factor(N);
    // long rows: 1024 threads, one butterfly per thread and stage
    if (N <= PD_LDS_ELEMS) {
        const int CBP = PD_LDS_ELEMS / N > 32 ? 32 : PD_LDS_ELEMS / N;
        const unsigned grid = (N + 2 * CBP - 1) / (2 * CBP);
        if (N == 1024)
            k_full_rows<PD_LDS_ELEMS, 1024, 1024><<<grid, 1024, 0, s>>>(
                cfull, stats, M, amax, tw, fr, CBP, window, (double2 *)B);
        else if (N >= 512)
            k_full_rows<PD_LDS_ELEMS, 1024><<<grid, 1024, 0, s>>>(cfull, stats, M, amax, tw, fr,
                                                                CBP, window, (double2 *)B);
        else
            k_full_rows<PD_LDS_ELEMS, FFT_THREADS><<<grid, FFT_THREADS, 0, s>>>(
                cfull, stats, M, amax, tw, fr, CBP, window, (double2 *)B);
    } else {
        k_full_rows<FFT_LDS_ELEMS, 1024><<<(N + 1) / 2, 1024, 0, s>>>(
            cfull, stats, M, amax, tw, fr, 1, window, (double2 *)B);
    }
    return hipGetLastError();
}

// The first three axes of an in-place N^4 DFT whose last axis is done
// (k_c5_lines transforms along it as it folds).
hipError_t launch_fft4_tail(double *Q, int N, const double2 *tw, hipStream_t s)
{
    double2 *d = (double2 *)Q;
    const FftRadices fr = factor(N);
    const int64_t N2 = (int64_t)N * N, N3 = N2 * N;
    fft_axis(d, tw, fr, N3, N, N, 1, N2, s);      // third
    fft_axis(d, tw, fr, N3, N2, N2, 1, N3, s);    // second
    fft_axis(d, tw, fr, N3, N3, N3, 1, 0, s);     // first
    return hipGetLastError();
}

// In-place DFTs along k1 of an N x N row-major complex array.
hipError_t launch_fft_cols(double *B, int N, const double2 *tw, hipStream_t s)
{
    fft_axis((double2 *)B, tw, factor(N), N, N, N, 1, 0, s);
    return hipGetLastError();
}

// Fold, window and m3 transforms of the trispectrum grid into T.
hipError_t launch_tri_lines(const double *c4, int M, int N, int window, const double2 *tw,
                            double *T, hipStream_t s)
{
    const FftRadices fr = factor(N);
    // line pairs per workgroup: what the LDS area holds, at most 32, and few
    // enough that the grid has about 512 workgroups
    const int64_t lines = (int64_t)N * N;
    int CBP = PD_LDS_ELEMS / N > 32 ? 32 : PD_LDS_ELEMS / N;
    const int64_t fill = lines / (2 * 512);
    if (fill < CBP)
        CBP = fill < 1 ? 1 : (int)fill;
    k_tri_lines<<<(unsigned)((lines + 2 * CBP - 1) / (2 * CBP)), FFT_THREADS, 0, s>>>(
        c4, M, tw, fr, CBP, window, (double2 *)T);
    return hipGetLastError();
}

// The k2 and k1 passes of an in-place N^3 DFT whose k3 pass is done.
hipError_t launch_fft3_tail(double *T, int N, const double2 *tw, hipStream_t s)
{
    double2 *d = (double2 *)T;
    const FftRadices fr = factor(N);
    const int64_t N2 = (int64_t)N * N;
    fft_axis(d, tw, fr, N2, N, N, 1, N2, s);     // axis 1
    fft_axis(d, tw, fr, N2, N2, N2, 1, 0, s);    // axis 0
    return hipGetLastError();
}

}  // namespace hos
