// hos_probe.hip -- the matrix cores' attainable rate on the device at hand.
//
// Not a step of the estimator: a measurement helper that puts a number on
// "the MFMA ceiling" the contractions are compared with.  One workgroup of
// four waves per compute unit (one wave per SIMD, the occupancy of the
// single-series contraction), each wave issuing `iters` rounds of four
// independent 32 x 32 matrix-core ops (four accumulators, no dependence
// between consecutive ops; iters is rounded up to even), nothing else in
// the loop.  Under that load the chip runs at its power-limited clock, so
// the rate is what a contraction could reach at best, below the published
// peak.
#include <type_traits>

#include <hip/hip_fp16.h>

#include "hos_internal.h"

namespace hos {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Operands: eight pseudo-random pairs per lane (uniform in [-1, 1), a
// counter-based hash of lane and index), cycled through by the ops, so the
// matrix cores see data as varied as a contraction's (the power the ops draw,
// and with it the clock, depends on how many operand bits toggle).  The
// accumulators are stored only when their sum equals `never` (the host
// passes NaN, which equals nothing), so the ops cannot be removed and
// nothing is written.
__device__ inline float probe_value(uint32_t lane, uint32_t j)
{
    uint32_t z = lane * 0x9e3779b9u + j * 0x85ebca6bu + 0x27d4eb2fu;
    z ^= z >> 15;
    z *= 0x2c1b3c6du;
    z ^= z >> 12;
    z *= 0x297a2d39u;
    z ^= z >> 15;
    return (float)(z >> 8) * 0x1p-23f - 1.0f;
}

template <int PATH>
__global__ void __launch_bounds__(256, 1)
k_probe_mfma(int32_t iters, float never, float *__restrict__ sink)
{
    const uint32_t lane = threadIdx.x + 256u * blockIdx.x;
    floatx16 c[4] = {};
    if constexpr (PATH == HOS_PATH_FP32) {
        float a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a[q] = probe_value(lane, 2 * q);
            b[q] = probe_value(lane, 2 * q + 1);
        }
        for (int32_t it = 0; it < iters; it += 2) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                c[q & 3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], b[q], c[q & 3], 0, 0, 0);
        }
    } else {
        typedef typename std::conditional<PATH == HOS_PATH_SPLIT_FP16, halfx8, bf16x8>::type vec;
        typedef typename std::conditional<PATH == HOS_PATH_SPLIT_FP16, _Float16, __bf16>::type el;
        vec a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[q][e] = (el)probe_value(lane, 16 * q + e);
                b[q][e] = (el)probe_value(lane, 16 * q + 8 + e);
            }
        for (int32_t it = 0; it < iters; it += 2) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if constexpr (PATH == HOS_PATH_SPLIT_FP16)
                    c[q & 3] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[q], b[q], c[q & 3], 0, 0, 0);
                else
                    c[q & 3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q], b[q], c[q & 3], 0, 0, 0);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v)
        s += c[0][v] + c[1][v] + c[2][v] + c[3][v];
    if (s == never)
        sink[lane] = s;
}

}  // namespace
}  // namespace hos

using namespace hos;

extern "C" int hos_mfma_rate(int32_t path, int32_t iters, float *ms_out, double *flops_out,
                             hipStream_t stream)
{
    if (path != HOS_PATH_FP32 && path != HOS_PATH_SPLIT_FP16 && path != HOS_PATH_SPLIT_BF16)
        return HOS_EINVAL;
    if (iters < 1 || iters > (1 << 24) || !ms_out || !flops_out)
        return HOS_EINVAL;
    int st = device_ok_public();
    if (st != HOS_OK)
        return st;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return HOS_EDEVICE;
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess)
        return HOS_EDEVICE;
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return HOS_EDEVICE;
    }
    const float never = __builtin_nanf("");
    auto launch = [&](int32_t n) {
        if (path == HOS_PATH_FP32)
            k_probe_mfma<HOS_PATH_FP32><<<cus, 256, 0, stream>>>(n, never, nullptr);
        else if (path == HOS_PATH_SPLIT_FP16)
            k_probe_mfma<HOS_PATH_SPLIT_FP16><<<cus, 256, 0, stream>>>(n, never, nullptr);
        else
            k_probe_mfma<HOS_PATH_SPLIT_BF16><<<cus, 256, 0, stream>>>(n, never, nullptr);
        return hipGetLastError();
    };
    // a short warm-up brings the clocks to their loaded state
    hipError_t e = launch(iters / 8 + 1);
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    if (e == hipSuccess) e = launch(iters);
    if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (e != hipSuccess)
        return HOS_EDEVICE;
    const double per_op = path == HOS_PATH_FP32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
    *ms_out = ms;
    const double rounds = (double)((iters + 1) & ~1);
    *flops_out = (double)cus * 4 /* waves */ * 4 /* ops per round */ * rounds * per_op;
    return HOS_OK;
}
