// k_batch.hip -- per-series finishing of a batch: c3 output, window + fold
// onto the DFT grid, the 2-D DFTs (one batched transform per DFT size), the
// principal-domain gather, and the bispectrum-matching loss.
//
// Principal domain (Algorithm DBS step 4, on the N grid): 0 <= k2 <= k1 and
// k1 + k2 < N/2, i.e. k1 + k2 <= H = floor((N-1)/2).  Its points are stored
// in row-major order (k1, then k2): row k1 holds min(k1, H - k1) + 1 points.
#include "hos_internal.h"
#include "hos_device.h"

namespace hos {

namespace {

__device__ inline int pd_row_len(int k1, int H) { return k1 <= H ? min(k1, H - k1) + 1 : 0; }

// (k1, k2) of principal-domain point p.
__device__ inline void pd_point(int p, int N, int &k1, int &k2)
{
    const int H = (N - 1) / 2;
    int a = 0;
    while (p >= pd_row_len(a, H)) {
        p -= pd_row_len(a, H);
        ++a;
    }
    k1 = a;
    k2 = p;
}

// Index of (k1, k2) in the principal domain, or -1 outside it.
__device__ inline int pd_index(int k1, int k2, int N)
{
    const int H = (N - 1) / 2;
    if (k2 > k1 || k1 + k2 > H)
        return -1;
    int p = 0;
    for (int a = 0; a < k1; ++a)
        p += pd_row_len(a, H);
    return p + k2;
}

__global__ void __launch_bounds__(256)
k_bc3_out(const SeriesDesc *__restrict__ sd, const char *__restrict__ ws, double *__restrict__ c3)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int side = 2 * d.M + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)side * side)
        return;
    const char *r = ws + d.ws_off;
    const double *stats = (const double *)(r + d.o_stats);
    const int w1 = (int)(idx / side) - d.M, w2 = (int)(idx % side) - d.M;
    c3[d.c3_off + idx] = c3_from_table((const double *)(r + d.o_cfull), d.M, stats[3], w1, w2);
}

// grid[m1][m2] = (sum over lags w = m mod N of W3(w) c3(w), 0)
__global__ void __launch_bounds__(256)
k_bfold(const SeriesDesc *__restrict__ sd, char *__restrict__ ws, int window)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int N = d.N, M = d.M;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N)
        return;
    const char *r = ws + d.ws_off;
    const double *cfull = (const double *)(r + d.o_cfull);
    const double norm = ((const double *)(r + d.o_stats))[3];
    const int m1 = (int)(idx / N), m2 = (int)(idx % N);
    double sum = 0.0;
    for (int w1 = m1 - N; w1 <= m1; w1 += N) {
        if (w1 < -M || w1 > M)
            continue;
        for (int w2 = m2 - N; w2 <= m2; w2 += N) {
            if (w2 < -M || w2 > M)
                continue;
            sum += window3(w1, w2, M, window == HOS_WIN_PARZEN) *
                   c3_from_table(cfull, M, norm, w1, w2);
        }
    }
    ((double2 *)(ws + d.grid_off))[idx] = make_double2(sum, 0.0);
}

__global__ void __launch_bounds__(256)
k_bpd(const SeriesDesc *__restrict__ sd, const char *__restrict__ ws, double2 *__restrict__ B_pd)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.npd)
        return;
    int k1, k2;
    pd_point(p, d.N, k1, k2);
    B_pd[d.pd_off + p] = ((const double2 *)(ws + d.grid_off))[(int64_t)k1 * d.N + k2];
}

// Per-series sum over the principal domain of |B - target|^2 (fixed order).
__global__ void __launch_bounds__(256)
k_bloss(const SeriesDesc *__restrict__ sd, const double2 *__restrict__ B_pd,
        const double2 *__restrict__ target, double *__restrict__ part)
{
    __shared__ double red[256];
    const SeriesDesc &d = sd[blockIdx.x];
    double s = 0.0;
    for (int p = threadIdx.x; p < d.npd; p += 256) {
        const double2 b = B_pd[d.pd_off + p], t = target[p];
        const double re = b.x - t.x, im = b.y - t.y;
        s += re * re + im * im;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
k_bloss_final(const double *__restrict__ part, int batch, double *__restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < batch; b += 256)
        s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[0] = red[0];
}

}  // namespace

hipError_t launch_batch_spectra(const BatchHeader &h, const char *dplan, int window, double *c3,
                                double *B_pd, char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    const int B = (int)h.batch;
    if (c3)
        k_bc3_out<<<dim3((unsigned)((h.max_side2 + 255) / 256), B), 256, 0, s>>>(sd, ws, c3);
    if (B_pd) {
        const int64_t n2 = h.max_N * h.max_N;
        k_bfold<<<dim3((unsigned)((n2 + 255) / 256), B), 256, 0, s>>>(sd, ws, window);
        // the group table is read on the host from the host copy of the plan
        const FftGroup *groups = (const FftGroup *)((const char *)&h + h.groups_off);
        for (int g = 0; g < (int)h.n_groups; ++g) {
            const FftGroup &gr = groups[g];
            double2 *tw = (double2 *)(ws + gr.twid_off);
            hipError_t e = launch_twiddles(tw, gr.N, s);
            if (e == hipSuccess)
                e = launch_fft2_batch((double *)(ws + gr.grid_off), gr.N, gr.count, tw, s);
            if (e != hipSuccess)
                return e;
        }
        k_bpd<<<dim3((unsigned)((h.max_npd + 255) / 256), B), 256, 0, s>>>(sd, ws,
                                                                         (double2 *)B_pd);
    }
    return hipGetLastError();
}

hipError_t launch_batch_loss(const BatchHeader &h, const char *dplan, const double *B_pd,
                             const double *target, double *loss, char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    double *part = (double *)(ws + h.loss_off);
    k_bloss<<<(unsigned)h.batch, 256, 0, s>>>(sd, (const double2 *)B_pd,
                                              (const double2 *)target, part);
    k_bloss_final<<<1, 256, 0, s>>>(part, (int)h.batch, loss);
    return hipGetLastError();
}

}  // namespace hos
