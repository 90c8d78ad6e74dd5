// k_finish.hip -- normalisation, mirroring and lag window of c3.
//
// C[a][b] (0 <= b <= a <= M) holds the scaled third-order sums over the
// fundamental region.  For a lag pair (w1, w2) the three sample offsets
// {0, w1, w2}, shifted by their minimum and sorted, are {0, b, a}; because
// the sum runs over every t with all indices inside the record, shifting
// t by that minimum maps c3(w1, w2) exactly onto C[a][b] / (n s^3) -- this
// is the six-fold symmetry of c3, used here only to relabel.  The table's
// lower triangle covers the hexagon; its upper triangle, when computed, the
// square's two corners (spans M < a <= 2M).  c3 is written on the hexagon
// (corners 0) or on the whole square.
//
// The lag window replaces the paper's frequency-domain box smoothing
// (Algorithm DBS's box smoothing): W3(w1,w2) = d(w1) d(w2) d(w1-w2) with the Parzen
// d and scale L = M.  The windowed cumulant is folded onto the N x N DFT
// grid (index w mod N; aliased lags add), which makes the grid DFT equal
// to sum_w W3(w) c3(w) exp(-2 pi i <k,w>/N) exactly; the fold happens inside
// the row-transform kernel (k_full_rows, k_fft.hip), which never writes the
// real grid.
#include "hos_internal.h"
#include "hos_device.h"

namespace hos {

namespace {

__global__ void __launch_bounds__(256)
k_c3_out(const double *__restrict__ cfull, const double *__restrict__ stats, int M, int amax,
         double *__restrict__ c3)
{
    const int side = 2 * M + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)side * side)
        return;
    const int w1 = (int)(idx / side) - M, w2 = (int)(idx % side) - M;
    c3[idx] = c3_from_table(cfull, M, amax, stats[3], w1, w2);
}

// Principal domain 0 <= k2 <= k1, k1 + k2 <= H = floor((N-1)/2) of the grid,
// packed row-major.  Row k1 holds min(k1, H - k1) + 1 points: k1 + 1 up to
// h = floor(H / 2), H - k1 + 1 after, so the rows before k1 hold
// p(p+1)/2 points (p = min(k1, h+1)) plus, past h + 1, the falling rows'
// sum.  One thread per grid point of the rows k1 <= H.
__global__ void __launch_bounds__(256)
k_pd_gather(const double2 *__restrict__ B, int N, double2 *__restrict__ out)
{
    const int H = (N - 1) / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(H + 1) * N)
        return;
    const int k1 = (int)(idx / N), k2 = (int)(idx % N);
    if (k2 > k1 || k1 + k2 > H)
        return;
    const int64_t h = H / 2;
    const int64_t p = k1 < h + 1 ? k1 : h + 1;
    int64_t start = p * (p + 1) / 2;
    if (k1 > h + 1)
        start += (int64_t)(k1 - h - 1) * (H + 1) - ((int64_t)(k1 - 1) * k1 / 2 - h * (h + 1) / 2);
    out[start + k2] = B[(int64_t)k1 * N + k2];
}

}  // namespace

// c3 and the row transforms of B from a reduced table (stats[3] divides it).
hipError_t launch_c3_finish_table(const double *cfull, const double *stats, int M, int amax,
                                  int window, int nfft, const double2 *tw, double *c3,
                                  int c3_amax, double *B, hipStream_t s)
{
    if (c3) {
        const int64_t tot = (int64_t)(2 * M + 1) * (2 * M + 1);
        k_c3_out<<<(tot + 255) / 256, 256, 0, s>>>(cfull, stats, M,
                                                   c3_amax < amax ? c3_amax : amax, c3);
    }
    if (B) {   // fold + window + row transforms (k_fft.hip); the columns follow
        hipError_t e = launch_full_rows(cfull, stats, M, amax, nfft, window, tw, B, s);
        if (e != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

hipError_t launch_c3_finish(const C3Plan &p, int window, int nfft, double *c3, int c3_amax,
                            double *B, char *ws, hipStream_t s)
{
    return launch_c3_finish_table((const double *)(ws + p.off_cfull),
                                  (const double *)(ws + p.off_stats), p.M, p.amax, window, nfft,
                                  (const double2 *)(ws + p.off_twid), c3, c3_amax, B, s);
}

hipError_t launch_pd_gather(const double *B, int N, double *B_pd, hipStream_t s)
{
    const int64_t tot = (int64_t)((N - 1) / 2 + 1) * N;
    k_pd_gather<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const double2 *)B, N,
                                                              (double2 *)B_pd);
    return hipGetLastError();
}

}  // namespace hos
