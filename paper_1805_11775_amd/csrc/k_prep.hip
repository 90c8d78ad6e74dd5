// k_prep.hip -- mean removal and operand preparation (FP64 on the way in).
//
// The estimator starts with Algorithm DBS's per-part mean removal, with the
// whole record as the one part (Section 4.1 uses K = 1).  The mean is a
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
    // MOM_BATCH loads go out together (past the end: sample 0, not summed);
    // the sums keep the one-sample order
    constexpr int MOM_BATCH = 8;
    for (int64_t t0 = (int64_t)blk * blockDim.x + threadIdx.x; t0 < n;
         t0 += MOM_BATCH * stride) {
        T v[MOM_BATCH];
#pragma unroll
        for (int u = 0; u < MOM_BATCH; ++u) {
            const int64_t t = t0 + u * stride;
            v[u] = x[t < n ? t : 0];
        }
#pragma unroll
        for (int u = 0; u < MOM_BATCH; ++u) {
            if (t0 + u * stride < n) {
                const double w = (double)v[u];
                sum += w;
                mn = fmin(mn, w);
                mx = fmax(mx, w);
            }
        }
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
// the sample's index in the whole record, key0 + o, so every table entry
// holding a sample agrees, in whichever piece of the record it is
// prepared); 0 outside the data.
template <typename T>
__device__ inline float centred(const T *__restrict__ x, int64_t n, int64_t o, double mu,
                                double s, int64_t key0)
{
    return (o >= 0 && o < n)
               ? round_stochastic_f32(((double)x[o] - mu) * s, (uint64_t)(key0 + o))
               : 0.0f;
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

// Table entries [o0, o0 + 256) of one workgroup (entries past oend are not
// written): the 263 samples they touch are rounded once into LDS, then every
// table is written from there.  MODE 0: xf and win4; 1/2: also the FP16/BF16
// hi|lo window tables.  xf -- the first factor x_i of every product -- is 0
// from nfirst on, so a piece of a record (its samples plus the following
// M as a halo) sums exactly over its own i while the window tables reach
// into the halo; nfirst = n for a whole record.
template <typename T, int MODE>
__device__ inline void prep_block(const T *__restrict__ x, int64_t n, int64_t o0, int64_t oend,
                                  const double *__restrict__ stats, float *__restrict__ xf,
                                  float4 *__restrict__ win4, uint4 *__restrict__ win8h,
                                  uint4 *__restrict__ win8l, int64_t key0 = 0,
                                  int64_t nfirst = INT64_MAX)
{
    __shared__ float sv[256 + 8];
    const double mu = stats[0], s = stats[1];
    const int t = threadIdx.x;
    sv[t] = centred(x, n, o0 + t, mu, s, key0);
    if (t < 8)
        sv[256 + t] = centred(x, n, o0 + 256 + t, mu, s, key0);
    __syncthreads();
    const int64_t o = o0 + t;
    if (o >= oend)
        return;
    // the tables are written once and read by another kernel: streaming
    // (nontemporal) stores
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x4n __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(o < nfirst ? sv[t] : 0.0f, xf + o);
    __builtin_nontemporal_store(f32x4{sv[t], sv[t + 1], sv[t + 2], sv[t + 3]},
                                (f32x4 *)(win4 + o));
    if constexpr (MODE != 0) {
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            uint16_t h0, l0, h1, l1;
            if (MODE == 2) {
                splitbf(sv[t + e], h0, l0);
                splitbf(sv[t + e + 1], h1, l1);
            } else {
                split16(sv[t + e], h0, l0);
                split16(sv[t + e + 1], h1, l1);
            }
            hw[e / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
            lw[e / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
        }
        __builtin_nontemporal_store(u32x4n{hw[0], hw[1], hw[2], hw[3]}, (u32x4n *)(win8h + o));
        __builtin_nontemporal_store(u32x4n{lw[0], lw[1], lw[2], lw[3]}, (u32x4n *)(win8l + o));
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_prep(const T *__restrict__ x, int64_t n, int64_t npad,
                                              const double *__restrict__ stats,
                                              float *__restrict__ xf, float4 *__restrict__ win4,
                                              uint4 *__restrict__ win8h,
                                              uint4 *__restrict__ win8l, int64_t key0,
                                              int64_t nfirst)
{
    prep_block<T, MODE>(x, n, (int64_t)blockIdx.x * 256, npad, stats, xf, win4, win8h, win8l,
                        key0, nfirst);
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

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_bprep(const T *__restrict__ x,
                                               const SeriesDesc *__restrict__ sd,
                                               char *__restrict__ ws)
{
    const SeriesDesc &d = sd[blockIdx.y];
    const int64_t o0 = (int64_t)blockIdx.x * 256 - d.lpad;
    if (o0 >= d.npad)
        return;
    char *r = ws + d.ws_off;
    prep_block<T, MODE>(x + d.x_off, d.n, o0, d.npad, (const double *)(r + d.o_stats),
                        (float *)(r + d.o_xf), (float4 *)(r + d.o_win4),
                        (uint4 *)(r + d.o_win8h), (uint4 *)(r + d.o_win8l));
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
        k_bprep<T, 0><<<grid, 256, 0, s>>>(x, sd, ws);
    else if (h.path == HOS_PATH_SPLIT_FP16)
        k_bprep<T, 1><<<grid, 256, 0, s>>>(x, sd, ws);
    else
        k_bprep<T, 2><<<grid, 256, 0, s>>>(x, sd, ws);
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

template <typename T>
void launch_prep_t(const T *x, const SeriesPlan &p, char *ws, hipStream_t s, int64_t key0,
                   int64_t nfirst)
{
    const double *stats = (const double *)(ws + p.off_stats);
    float *xf = (float *)(ws + p.off_xf);
    float4 *win4 = (float4 *)(ws + p.off_win4);
    uint4 *h = (uint4 *)(ws + p.off_win8h), *l = (uint4 *)(ws + p.off_win8l);
    const int64_t blocks = (p.npad + 255) / 256;
    if (p.path == HOS_PATH_FP32)
        k_prep<T, 0><<<blocks, 256, 0, s>>>(x, p.n, p.npad, stats, xf, win4, h, l, key0, nfirst);
    else if (p.path == HOS_PATH_SPLIT_FP16)
        k_prep<T, 1><<<blocks, 256, 0, s>>>(x, p.n, p.npad, stats, xf, win4, h, l, key0, nfirst);
    else
        k_prep<T, 2><<<blocks, 256, 0, s>>>(x, p.n, p.npad, stats, xf, win4, h, l, key0, nfirst);
}

hipError_t launch_prep(const void *x, int dtype, const SeriesPlan &p, char *ws, hipStream_t s,
                       int64_t key0, int64_t nfirst)
{
    if (nfirst < 0)
        nfirst = p.n;
    if (dtype == HOS_F64)
        launch_prep_t<double>((const double *)x, p, ws, s, key0, nfirst);
    else
        launch_prep_t<float>((const float *)x, p, ws, s, key0, nfirst);
    return hipGetLastError();
}

// Streaming: fold one piece's block partials (sum, min, max) into the
// running totals acc (3 doubles), in piece order; first = 1 starts them.
__global__ void __launch_bounds__(64)
k_mom_accumulate(const double *__restrict__ part, int nblk, int first, double *__restrict__ acc)
{
    if (threadIdx.x != 0)
        return;
    double sum = 0.0, mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int b = 0; b < nblk; ++b) {
        sum += part[3 * b];
        mn = fmin(mn, part[3 * b + 1]);
        mx = fmax(mx, part[3 * b + 2]);
    }
    if (first) {
        acc[0] = sum;
        acc[1] = mn;
        acc[2] = mx;
    } else {
        acc[0] += sum;
        acc[1] = fmin(acc[1], mn);
        acc[2] = fmax(acc[2], mx);
    }
}

hipError_t launch_moments_piece(const void *x, int dtype, int64_t len, int first,
                                const SeriesPlan &p, char *ws, double *acc, hipStream_t s)
{
    double *part = (double *)(ws + p.off_mpart);
    if (dtype == HOS_F64)
        k_moments_partial<double><<<MOM_BLOCKS, 256, 0, s>>>((const double *)x, len, part);
    else
        k_moments_partial<float><<<MOM_BLOCKS, 256, 0, s>>>((const float *)x, len, part);
    k_mom_accumulate<<<1, 64, 0, s>>>(part, MOM_BLOCKS, first, acc);
    return hipGetLastError();
}

// The statistics of the whole record from the running totals.
hipError_t launch_moments_total(const double *acc, int64_t n, uint32_t flags, int top,
                                double *stats, hipStream_t s)
{
    k_moments_final<<<1, 256, 0, s>>>(acc, 1, n, flags, top, stats);
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
