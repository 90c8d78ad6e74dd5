// k_batch.hip -- per-series finishing of a batch: the c3 output, the
// principal-domain spectra (k_fft.hip) and the bispectrum-matching loss.
//
// Principal domain (Algorithm DBS's raw bispectrum, on the N grid): 0 <= k2 <= k1 and
// k1 + k2 < N/2, i.e. k1 + k2 <= H = floor((N-1)/2).  Its points are stored
// in row-major order (k1, then k2): row k1 holds min(k1, H - k1) + 1 points.
#include "hos_internal.h"
#include "hos_device.h"

namespace hos {

namespace {

__device__ inline int pd_row_len(int k1, int H) { return k1 <= H ? min(k1, H - k1) + 1 : 0; }

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
    c3[d.c3_off + idx] = c3_from_table((const double *)(r + d.o_cfull), d.M, d.M, stats[3], w1, w2);
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

// Segment averaging: entry e of the reduced tables of every series (each
// divided by its own n s^3), summed in series order and divided by the
// number of series; stats[3] = 1 then makes the average the table that the
// single-series finishing kernels read.
__global__ void __launch_bounds__(256)
k_seg_avg(const SeriesDesc *__restrict__ sd, int64_t S, int M, const char *__restrict__ ws,
          double *__restrict__ avg, double *__restrict__ stats)
{
    const int64_t ne = (int64_t)(M + 1) * (M + 1);
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < 64)
        stats[threadIdx.x] = threadIdx.x == 3 ? 1.0 : 0.0;
    if (e >= ne)
        return;
    double s = 0.0;
    for (int64_t i = 0; i < S; ++i) {
        const char *r = ws + sd[i].ws_off;
        s += ((const double *)(r + sd[i].o_cfull))[e] / ((const double *)(r + sd[i].o_stats))[3];
    }
    avg[e] = s / (double)S;
}

}  // namespace

hipError_t launch_seg_average(const BatchHeader &h, const char *dplan, char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    const int M = (int)h.uniform_M;
    const int64_t ne = (int64_t)(M + 1) * (M + 1);
    double *avg = (double *)(ws + h.seg_off);
    double *stats = avg + ne;
    k_seg_avg<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(sd, h.batch, M, ws, avg, stats);
    return hipGetLastError();
}

hipError_t launch_batch_spectra(const BatchHeader &h, const char *dplan, int window, double *c3,
                                double *B_pd, char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    const int B = (int)h.batch;
    if (c3)
        k_bc3_out<<<dim3((unsigned)((h.max_side2 + 255) / 256), B), 256, 0, s>>>(sd, ws, c3);
    if (B_pd) {
        hipError_t e = launch_pd_spectra(h, dplan, window, ws, B_pd, s);
        if (e != hipSuccess)
            return e;
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
