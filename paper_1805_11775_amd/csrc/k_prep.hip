// k_prep.hip -- mean removal and operand preparation (FP64 on the way in).
//
// Step 1 of the estimator is the mean removal of Algorithm DBS step 2, with
// the whole record as the one part (Section 4.1 uses K = 1).  The mean is a
// fixed-order FP64 reduction.  The centred series is then multiplied by an
// exact power of two s that puts max|x~ s| in [2^(top-1), 2^top): [64, 128)
// for the third order and [16, 32) for the fourth, which keeps every FP16
// product row (x~ x~, resp. x~ x~ x~, below 2^15) inside the FP16 range.  The
// factor is divided out exactly (as s^2, s^3 or s^4) when the cumulant is
// normalised.
//
// Operand tables written for the contraction (n_pad >= n, zero beyond n):
//   xf[o]    = float(x~_o s), stochastically rounded  plain FP32 series
//   win4[o]  = (xf[o], xf[o+1], xf[o+2], xf[o+3])  16-byte window table
//   win8h[o] = (hi[o] .. hi[o+7]),  win8l[o] = (lo[o] .. lo[o+7])
// where hi = RNE16(xf), lo = RNE16(xf - hi) in FP16 or BF16.  The window
// tables let every lane fetch 4 floats or 8 halves starting at ANY sample
// with one aligned 16-byte load (the Hankel operand x_{i+b} starts at a
// different sample in every lane).
#include "hos_internal.h"
#include "hos_device.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace hos {

namespace {

// Sum, min and max of x over the samples t = blk*256 + tid (stride nblk*256).
template <typename T>
__device__ inline void moments_partial_body(const T *__restrict__ x, int64_t n, int blk,
                                            int nblk, double *__restrict__ part)
{
    __shared__ double s_sum[256], s_min[256], s_max[256];
    double sum = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t t = (int64_t)blk * blockDim.x + threadIdx.x; t < n; t += stride) {
        double v = (double)x[t];
        sum += v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    const int tid = threadIdx.x;
    s_sum[tid] = sum;
    s_min[tid] = mn;
    s_max[tid] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            s_sum[tid] += s_sum[tid + w];
            s_min[tid] = fmin(s_min[tid], s_min[tid + w]);
            s_max[tid] = fmax(s_max[tid], s_max[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[3 * blk + 0] = s_sum[0];
        part[3 * blk + 1] = s_min[0];
        part[3 * blk + 2] = s_max[0];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_moments_partial(const T *__restrict__ x,
                                                         int64_t n,
                                                         double *__restrict__ part)
{
    moments_partial_body(x, n, blockIdx.x, gridDim.x, part);
}

// Combines nblk <= 256 block partials (fixed-order tree, one per thread) into
// stats[0] = mean removed, stats[1] = scale s, stats[2] = max|x~|,
// stats[3] = n s^3, stats[4] = n s^4 (exact: s is a power of two).
__device__ inline void moments_final_body(const double *__restrict__ part, int nblk, int64_t n,
                                          uint32_t flags, int top, double *__restrict__ stats)
{
    __shared__ double s_sum[256], s_min[256], s_max[256];
    const int tid = threadIdx.x;
    const bool on = tid < nblk;
    s_sum[tid] = on ? part[3 * tid + 0] : 0.0;
    s_min[tid] = on ? part[3 * tid + 1] : __builtin_huge_val();
    s_max[tid] = on ? part[3 * tid + 2] : -__builtin_huge_val();
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            s_sum[tid] += s_sum[tid + w];
            s_min[tid] = fmin(s_min[tid], s_min[tid + w]);
            s_max[tid] = fmax(s_max[tid], s_max[tid + w]);
        }
        __syncthreads();
    }
    if (tid != 0)
        return;
    const double sum = s_sum[0], mn = s_min[0], mx = s_max[0];
    double mu = (flags & HOS_NO_CENTER) ? 0.0 : sum / (double)n;
    double amax = fmax(mx - mu, mu - mn);
    double s = 1.0;
    if (amax > 0.0 && isfinite(amax)) {
        int e;
        frexp(amax, &e);          // amax = m 2^e, m in [0.5, 1)
        s = ldexp(1.0, top - e);  // amax * s in [2^(top-1), 2^top)
    }
    stats[0] = mu;
    stats[1] = s;
    stats[2] = amax;
    stats[3] = (double)n * s * s * s;
    stats[4] = (double)n * s * s * s * s;
}

__global__ void __launch_bounds__(256) k_moments_final(const double *__restrict__ part,
                                                       int nblk, int64_t n, uint32_t flags,
                                                       int top, double *__restrict__ stats)
{
    moments_final_body(part, nblk, n, flags, top, stats);
}

// (x_o - mean) s formed in FP64 and rounded stochastically to FP32 (keyed by
// the sample index, so every table entry holding sample o agrees); 0 outside
// the record.
template <typename T>
__device__ inline float centred(const T *__restrict__ x, int64_t n, int64_t o, double mu,
                                double s)
{
    return (o >= 0 && o < n) ? round_stochastic_f32(((double)x[o] - mu) * s, (uint64_t)o)
                             : 0.0f;
}

// Table entry o (o < 0 is left padding): xf[o] and win4[o].
template <typename T>
__device__ inline void prep_f32_body(const T *__restrict__ x, int64_t n, int64_t o,
                                     const double *__restrict__ stats, float *__restrict__ xf,
                                     float4 *__restrict__ win4)
{
    const double mu = stats[0], s = stats[1];
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        v[e] = centred(x, n, o + e, mu, s);
    xf[o] = v[0];
    win4[o] = make_float4(v[0], v[1], v[2], v[3]);
}

__device__ inline void split16(float v, uint16_t &h, uint16_t &l)
{
    _Float16 hh = (_Float16)v;
    _Float16 ll = (_Float16)(v - (float)hh);
    h = __builtin_bit_cast(uint16_t, hh);
    l = __builtin_bit_cast(uint16_t, ll);
}

__device__ inline void splitbf(float v, uint16_t &h, uint16_t &l)
{
    __bf16 hh = (__bf16)v;
    __bf16 ll = (__bf16)(v - (float)hh);
    h = __builtin_bit_cast(uint16_t, hh);
    l = __builtin_bit_cast(uint16_t, ll);
}

// Table entry o: win8h[o], win8l[o] (8 halves each).
template <typename T, bool BF16>
__device__ inline void prep_split_body(const T *__restrict__ x, int64_t n, int64_t o,
                                       const double *__restrict__ stats,
                                       uint4 *__restrict__ win8h, uint4 *__restrict__ win8l)
{
    const double mu = stats[0], s = stats[1];
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        uint16_t h0, l0, h1, l1;
        float v0 = centred(x, n, o + e, mu, s), v1 = centred(x, n, o + e + 1, mu, s);
        if (BF16) {
            splitbf(v0, h0, l0);
            splitbf(v1, h1, l1);
        } else {
            split16(v0, h0, l0);
            split16(v1, h1, l1);
        }
        hw[e / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
        lw[e / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    win8h[o] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    win8l[o] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// One thread per table entry o of [0, npad).
template <typename T>
__global__ void __launch_bounds__(256) k_prep_f32(const T *__restrict__ x, int64_t n,
                                                  int64_t npad,
                                                  const double *__restrict__ stats,
                                                  float *__restrict__ xf,
                                                  float4 *__restrict__ win4)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < npad)
        prep_f32_body(x, n, o, stats, xf, win4);
}

template <typename T, bool BF16>
__global__ void __launch_bounds__(256) k_prep_split(const T *__restrict__ x, int64_t n,
                                                    int64_t npad,
                                                    const double *__restrict__ stats,
                                                    uint4 *__restrict__ win8h,
                                                    uint4 *__restrict__ win8l)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < npad)
        prep_split_body<T, BF16>(x, n, o, stats, win8h, win8l);
}

// ------------------------------------------------------------------ batches
// blockIdx.y = series; its descriptor gives the sample range and the
// workspace region.
template <typename T>
__global__ void __launch_bounds__(256) k_bmoments_partial(const T *__restrict__ x,
                                                          const SeriesDesc *__restrict__ sd,
                                                          char *__restrict__ ws)
{
    const SeriesDesc &d = sd[blockIdx.y];
    moments_partial_body(x + d.x_off, d.n, blockIdx.x, gridDim.x,
                         (double *)(ws + d.ws_off + d.o_mpart));
}

__global__ void __launch_bounds__(256) k_bmoments_final(const SeriesDesc *__restrict__ sd,
                                                        char *__restrict__ ws, int nblk,
                                                        uint32_t flags, int top)
{
    const SeriesDesc &d = sd[blockIdx.x];
    char *r = ws + d.ws_off;
    moments_final_body((const double *)(r + d.o_mpart), nblk, d.n, flags, top,
                       (double *)(r + d.o_stats));
}

template <typename T, int PATH>
__global__ void __launch_bounds__(256) k_bprep(const T *__restrict__ x,
                                               const SeriesDesc *__restrict__ sd,
                                               char *__restrict__ ws)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - d.lpad;
    if (o >= d.npad)
        return;
    char *r = ws + d.ws_off;
    const T *xs = x + d.x_off;
    const double *stats = (const double *)(r + d.o_stats);
    prep_f32_body(xs, d.n, o, stats, (float *)(r + d.o_xf), (float4 *)(r + d.o_win4));
    if constexpr (PATH != HOS_PATH_FP32)
        prep_split_body<T, PATH == HOS_PATH_SPLIT_BF16>(xs, d.n, o, stats,
                                                       (uint4 *)(r + d.o_win8h),
                                                       (uint4 *)(r + d.o_win8l));
}

template <typename T>
void launch_bprep_t(const T *x, const BatchHeader &h, const SeriesDesc *sd, char *ws,
                    hipStream_t s)
{
    const int B = (int)h.batch;
    k_bmoments_partial<T><<<dim3((unsigned)h.momb, B), 256, 0, s>>>(x, sd, ws);
    k_bmoments_final<<<B, 256, 0, s>>>(sd, ws, (int)h.momb, (uint32_t)h.flags, 7);
    const dim3 grid((unsigned)((h.max_lpad + h.max_npad + 255) / 256), B);
    if (h.path == HOS_PATH_FP32)
        k_bprep<T, HOS_PATH_FP32><<<grid, 256, 0, s>>>(x, sd, ws);
    else if (h.path == HOS_PATH_SPLIT_FP16)
        k_bprep<T, HOS_PATH_SPLIT_FP16><<<grid, 256, 0, s>>>(x, sd, ws);
    else
        k_bprep<T, HOS_PATH_SPLIT_BF16><<<grid, 256, 0, s>>>(x, sd, ws);
}

}  // namespace

hipError_t launch_moments(const void *x, int dtype, int64_t n, uint32_t flags,
                          const SeriesPlan &p, char *ws, hipStream_t s)
{
    double *part = (double *)(ws + p.off_mpart);
    double *stats = (double *)(ws + p.off_stats);
    if (dtype == HOS_F64)
        k_moments_partial<double><<<MOM_BLOCKS, 256, 0, s>>>((const double *)x, n, part);
    else
        k_moments_partial<float><<<MOM_BLOCKS, 256, 0, s>>>((const float *)x, n, part);
    k_moments_final<<<1, 256, 0, s>>>(part, MOM_BLOCKS, n, flags, p.scale_top, stats);
    return hipGetLastError();
}

hipError_t launch_prep(const void *x, int dtype, const SeriesPlan &p, char *ws, hipStream_t s)
{
    const double *stats = (const double *)(ws + p.off_stats);
    float *xf = (float *)(ws + p.off_xf);
    float4 *win4 = (float4 *)(ws + p.off_win4);
    const int64_t blocks = (p.npad + 255) / 256;
    if (dtype == HOS_F64)
        k_prep_f32<double><<<blocks, 256, 0, s>>>((const double *)x, p.n, p.npad, stats, xf, win4);
    else
        k_prep_f32<float><<<blocks, 256, 0, s>>>((const float *)x, p.n, p.npad, stats, xf, win4);
    if (p.path != HOS_PATH_FP32) {
        uint4 *h = (uint4 *)(ws + p.off_win8h), *l = (uint4 *)(ws + p.off_win8l);
        const bool bf = p.path == HOS_PATH_SPLIT_BF16;
        if (dtype == HOS_F64) {
            if (bf)
                k_prep_split<double, true><<<blocks, 256, 0, s>>>((const double *)x, p.n, p.npad, stats, h, l);
            else
                k_prep_split<double, false><<<blocks, 256, 0, s>>>((const double *)x, p.n, p.npad, stats, h, l);
        } else {
            if (bf)
                k_prep_split<float, true><<<blocks, 256, 0, s>>>((const float *)x, p.n, p.npad, stats, h, l);
            else
                k_prep_split<float, false><<<blocks, 256, 0, s>>>((const float *)x, p.n, p.npad, stats, h, l);
        }
    }
    return hipGetLastError();
}

}  // namespace hos

namespace hos {

hipError_t launch_batch_prep(const void *x, int dtype, const BatchHeader &h, const char *dplan,
                             char *ws, hipStream_t s)
{
    const SeriesDesc *sd = (const SeriesDesc *)(dplan + h.series_off);
    if (dtype == HOS_F64)
        launch_bprep_t<double>((const double *)x, h, sd, ws, s);
    else
        launch_bprep_t<float>((const float *)x, h, sd, ws, s);
    return hipGetLastError();
}

}  // namespace hos
