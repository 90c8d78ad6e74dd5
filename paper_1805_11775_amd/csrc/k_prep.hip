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
//   xf[o]    = float(x~_o s)                       plain FP32 series
//   win4[o]  = (xf[o], xf[o+1], xf[o+2], xf[o+3])  16-byte window table
//   win8h[o] = (hi[o] .. hi[o+7]),  win8l[o] = (lo[o] .. lo[o+7])
// where hi = RNE16(xf), lo = RNE16(xf - hi) in FP16 or BF16.  The window
// tables let every lane fetch 4 floats or 8 halves starting at ANY sample
// with one aligned 16-byte load (the Hankel operand x_{i+b} starts at a
// different sample in every lane).
#include "hos_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace hos {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_moments_partial(const T *__restrict__ x,
                                                         int64_t n,
                                                         double *__restrict__ part)
{
    __shared__ double s_sum[256], s_min[256], s_max[256];
    double sum = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
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
        part[3 * blockIdx.x + 0] = s_sum[0];
        part[3 * blockIdx.x + 1] = s_min[0];
        part[3 * blockIdx.x + 2] = s_max[0];
    }
}

// stats[0] = mean removed, stats[1] = scale s, stats[2] = max|x~|,
// stats[3] = n s^3, stats[4] = n s^4 (exact: s is a power of two)
__global__ void __launch_bounds__(64) k_moments_final(const double *__restrict__ part,
                                                      int nblk, int64_t n, uint32_t flags,
                                                      int top, double *__restrict__ stats)
{
    if (threadIdx.x != 0)
        return;
    double sum = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int b = 0; b < nblk; ++b) {
        sum += part[3 * b + 0];
        mn = fmin(mn, part[3 * b + 1]);
        mx = fmax(mx, part[3 * b + 2]);
    }
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

template <typename T>
__device__ inline float centred(const T *__restrict__ x, int64_t n, int64_t o, double mu,
                                double s)
{
    return o < n ? (float)(((double)x[o] - mu) * s) : 0.0f;
}

// One thread per sample o of the padded range: writes xf[o] and win4[o].
template <typename T>
__global__ void __launch_bounds__(256) k_prep_f32(const T *__restrict__ x, int64_t n,
                                                  int64_t npad,
                                                  const double *__restrict__ stats,
                                                  float *__restrict__ xf,
                                                  float4 *__restrict__ win4)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= npad)
        return;
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

// One thread per sample o: win8h[o], win8l[o] (8 halves each).
template <typename T, bool BF16>
__global__ void __launch_bounds__(256) k_prep_split(const T *__restrict__ x, int64_t n,
                                                    int64_t npad,
                                                    const double *__restrict__ stats,
                                                    uint4 *__restrict__ win8h,
                                                    uint4 *__restrict__ win8l)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= npad)
        return;
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
    k_moments_final<<<1, 64, 0, s>>>(part, MOM_BLOCKS, n, flags, p.scale_top, stats);
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
