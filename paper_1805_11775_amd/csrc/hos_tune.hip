// hos_tune.hip -- the batch contraction's tile tuner, timed on the device.
//
// A batch plan gives every series one of two tile classes for its c3
// contraction: 2 x 2 or 4 x 4 matrix-core blocks (split paths; the FP32 path
// has 4 x 4 only).  Small tiles waste less of F's triangle at small M, large
// tiles reuse each product row over more columns and stage fewer windows
// per sample.  hos_tune measures both for every (maximum lag, length
// bucket): a synthetic batch of `series` series with lengths spread evenly
// over the bucket, a plan per candidate, the operand tables built once, and
// the contraction launch alone timed `reps` times with HIP events (the
// other stages do not depend on the tile); the median decides.
//
// Chunk length and waves per workgroup are not candidates: both tile
// classes stage 1024-sample chunks in 4-wave workgroups (the one-launch
// batch kernel's LDS layout fixes them), and the split of a tile's sample
// range into work items follows from the plan's balance rule.
#include <string.h>

#include <algorithm>
#include <vector>

#include "hos_internal.h"
#include "hos_device.h"

namespace hos {
namespace {

// Synthetic input: uniform on (-1, 1) from a counter-based generator
// (SplitMix64 of the sample index), deterministic.
__global__ void __launch_bounds__(256) k_tune_fill(float *__restrict__ x, int64_t n, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t z = splitmix64(seed + (uint64_t)i);
    x[i] = (float)((double)(z >> 11) * 0x1.0p-52 - 1.0);
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Lengths of the synthetic batch for bucket [lo, hi): evenly spread, each
// longer than M.
void tune_lengths(int64_t lo, int64_t hi, int32_t series, int32_t M, std::vector<int64_t> &n)
{
    n.resize(series);
    for (int32_t s = 0; s < series; ++s) {
        const int64_t v = lo + (hi - 1 - lo) * s / (series > 1 ? series - 1 : 1);
        n[s] = std::max<int64_t>(v, (int64_t)M + 2);
    }
}

int tune_candidates(int32_t path, int32_t *cand)
{
    if (path == HOS_PATH_FP32) {
        cand[0] = 4;
        return 1;
    }
    cand[0] = 2;
    cand[1] = 4;
    return 2;
}

struct TuneSizes {
    int64_t x_elems;   // largest synthetic batch
    size_t plan_bytes, ws_bytes, total;
};

int tune_check(int32_t path, const int32_t *Ms, int32_t nM, const int64_t *edges, int32_t nb,
               int32_t series, int32_t reps)
{
    if (path != HOS_PATH_FP32 && path != HOS_PATH_SPLIT_FP16 && path != HOS_PATH_SPLIT_BF16)
        return HOS_EINVAL;
    if (!Ms || !edges || nM < 1 || nM > 64 || nb < 1 || nb > 16 || series < 1 ||
        series > 4096 || reps < 1 || reps > 100)
        return HOS_EINVAL;
    for (int32_t j = 0; j < nb; ++j)
        if (edges[j] < 2 || edges[j + 1] <= edges[j] + 1 || edges[j + 1] > ((int64_t)1 << 24))
            return HOS_EINVAL;
    for (int32_t i = 0; i < nM; ++i)
        if (Ms[i] < 0 || Ms[i] > 1024 || (int64_t)Ms[i] + 2 >= edges[nb])
            return HOS_EINVAL;
    return HOS_OK;
}

int tune_sizes(int32_t path, const int32_t *Ms, int32_t nM, const int64_t *edges, int32_t nb,
               int32_t series, TuneSizes &t)
{
    memset(&t, 0, sizeof(t));
    int32_t cand[2];
    const int nc = tune_candidates(path, cand);
    std::vector<int64_t> n;
    for (int32_t i = 0; i < nM; ++i)
        for (int32_t j = 0; j < nb; ++j) {
            tune_lengths(edges[j], edges[j + 1], series, Ms[i], n);
            int64_t tot = 0;
            for (int64_t v : n)
                tot += v;
            t.x_elems = std::max(t.x_elems, tot);
            std::vector<int32_t> M(series, Ms[i]);
            for (int c = 0; c < nc; ++c) {
                std::vector<int32_t> tile(series, cand[c]);
                BatchHeader h;
                const int st = batch_plan(series, n.data(), M.data(), HOS_WIN_PARZEN, path, 0,
                                          tile.data(), nullptr, 0, &h);
                if (st != HOS_OK)
                    return st;
                t.plan_bytes = std::max(t.plan_bytes, (size_t)h.blob_bytes);
                t.ws_bytes = std::max(t.ws_bytes, (size_t)h.ws_bytes);
            }
        }
    t.total = al256((size_t)t.x_elems * sizeof(float)) + al256(t.plan_bytes) + t.ws_bytes;
    return HOS_OK;
}

}  // namespace
}  // namespace hos

using namespace hos;

extern "C" int hos_tune_workspace(int32_t path, const int32_t *Ms, int32_t nM,
                                  const int64_t *n_edges, int32_t nb, int32_t series,
                                  size_t *bytes)
{
    if (!bytes)
        return HOS_EINVAL;
    int st = tune_check(path, Ms, nM, n_edges, nb, series, 1);
    if (st != HOS_OK)
        return st;
    TuneSizes t;
    st = tune_sizes(path, Ms, nM, n_edges, nb, series, t);
    if (st != HOS_OK)
        return st;
    *bytes = t.total;
    return HOS_OK;
}

extern "C" int hos_tune(int32_t path, const int32_t *Ms, int32_t nM, const int64_t *n_edges,
                        int32_t nb, int32_t series, int32_t reps, void *ws, size_t ws_bytes,
                        int32_t *tile_out, float *ms_out, hipStream_t stream)
{
    int st = tune_check(path, Ms, nM, n_edges, nb, series, reps);
    if (st != HOS_OK)
        return st;
    if (!ws || ((uintptr_t)ws & 255) || !tile_out || !ms_out)
        return HOS_EINVAL;
    TuneSizes t;
    st = tune_sizes(path, Ms, nM, n_edges, nb, series, t);
    if (st != HOS_OK)
        return st;
    if (ws_bytes < t.total)
        return HOS_EWORKSPACE;
    st = device_ok_public();
    if (st != HOS_OK)
        return st;

    char *base = (char *)ws;
    float *x = (float *)base;
    char *dplan = base + al256((size_t)t.x_elems * sizeof(float));
    char *w = dplan + al256(t.plan_bytes);
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess)
        return HOS_EDEVICE;
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return HOS_EDEVICE;
    }
    int32_t cand[2];
    const int nc = tune_candidates(path, cand);
    hipError_t e = hipSuccess;
    std::vector<int64_t> n;
    std::vector<char> blob;
    std::vector<float> times;
    for (int32_t i = 0; i < nM && e == hipSuccess; ++i)
        for (int32_t j = 0; j < nb && e == hipSuccess; ++j) {
            tune_lengths(n_edges[j], n_edges[j + 1], series, Ms[i], n);
            int64_t tot = 0;
            for (int64_t v : n)
                tot += v;
            k_tune_fill<<<(unsigned)((tot + 255) / 256), 256, 0, stream>>>(
                x, tot, 0x243f6a8885a308d3ull + 1000003ull * (uint64_t)(i * 16 + j));
            std::vector<int32_t> M(series, Ms[i]);
            float best = -1.0f;
            int32_t pick = cand[nc - 1];
            for (int c = 0; c < 2; ++c)
                ms_out[((int64_t)i * nb + j) * 2 + c] = -1.0f;
            for (int c = 0; c < nc && e == hipSuccess; ++c) {
                std::vector<int32_t> tile(series, cand[c]);
                BatchHeader h;
                batch_plan(series, n.data(), M.data(), HOS_WIN_PARZEN, path, 0, tile.data(),
                           nullptr, 0, &h);
                blob.assign((size_t)h.blob_bytes + 8, 0);
                char *hp = blob.data() + ((8 - ((uintptr_t)blob.data() & 7)) & 7);
                batch_plan(series, n.data(), M.data(), HOS_WIN_PARZEN, path, 0, tile.data(), hp,
                           (size_t)h.blob_bytes, nullptr);
                e = hipMemcpyAsync(dplan, hp, (size_t)h.blob_bytes, hipMemcpyHostToDevice, stream);
                if (e == hipSuccess) e = launch_batch_prep(x, HOS_F32, h, dplan, w, stream);
                if (e == hipSuccess) e = launch_batch_contract(h, dplan, w, stream);   // warm-up
                times.clear();
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    e = hipEventRecord(ev[0], stream);
                    if (e == hipSuccess) e = launch_batch_contract(h, dplan, w, stream);
                    if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
                    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                    float ms = 0.0f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                    times.push_back(ms);
                }
                // the host copy of the plan must outlive the copy: wait for it
                if (e == hipSuccess) e = hipStreamSynchronize(stream);
                if (e != hipSuccess)
                    break;
                std::sort(times.begin(), times.end());
                const float med = times[times.size() / 2];
                ms_out[((int64_t)i * nb + j) * 2 + (cand[c] == 4 ? 1 : 0)] = med;
                if (best < 0.0f || med < best) {
                    best = med;
                    pick = cand[c];
                }
            }
            tile_out[(int64_t)i * nb + j] = pick;
        }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}
