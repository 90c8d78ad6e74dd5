// Host-only exercise of the library's C ABI for the address and
// undefined-behaviour sanitizers: every planner, workspace query and
// argument check that runs before the first HIP call, over a deterministic
// sweep of sizes (edges, maxima, degenerate cases), with every output
// array sized exactly as documented so that an overrun is reported.  No
// call here reaches a device.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "hos.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64()
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static void c3_plans()
{
    const int paths[3] = {HOS_PATH_FP32, HOS_PATH_SPLIT_FP16, HOS_PATH_SPLIT_BF16};
    for (int k = 0; k < 60; ++k) {
        const int64_t n = k < 6 ? (int64_t[]){2, 3, 1024, 1025, 1 << 20, 70001}[k] : uniform(2, 300000);
        const int32_t M = (int32_t)uniform(0, n - 1 < 1500 ? n - 1 : 1500);
        const int path = paths[k % 3];
        int64_t info[10];
        CHECK(hos_c3_plan_info(n, M, path, info, 10) == HOS_OK);
        const int64_t TR = info[2], C = info[3];
        const int64_t cap = TR * (TR + 1) / 2 * C;
        if (cap > 0 && cap < (1 << 22)) {
            std::vector<int64_t> owner(cap), slot(cap), rslot(cap);
            CHECK(hos_c3_schedule(n, M, path, owner.data(), slot.data(), rslot.data(), cap) ==
                  HOS_OK);
            for (int64_t i = 0; i < cap; ++i)
                CHECK(owner[i] >= 0 && slot[i] == rslot[i]);
        }
        for (uint32_t flags : {0u, (uint32_t)HOS_FULL_SQUARE, (uint32_t)HOS_PD_ONLY}) {
            size_t b = 0;
            const int32_t nfft = M > 0 ? 2 * M : 2;
            const int st = hos_bispectrum_workspace(n, M, nfft, path, flags, &b);
            CHECK(st == HOS_OK || st == HOS_EINVAL);   // nfft need not be 2,3,5-smooth
        }
    }
}

static void high_order_plans()
{
    for (int k = 0; k < 40; ++k) {
        const int64_t n = uniform(200, 500000);
        const int32_t M4 = (int32_t)uniform(0, 127), M5 = (int32_t)uniform(0, 40);
        int64_t info[16];
        CHECK(hos_c4_plan_info(n, M4, k % 3, info, 16) == HOS_OK || M4 >= n);
        CHECK(hos_c5_plan_info(n, M5, k % 3, info, 16) == HOS_OK || M5 >= n);
        size_t b = 0;
        hos_trispectrum_workspace(n, M4, 0, k % 3, 0, &b);
        hos_cumulant5_workspace(n, M5, 0, k % 3, 0, &b);
    }
}

static void batch_plans()
{
    for (int k = 0; k < 30; ++k) {
        const int32_t batch = (int32_t)uniform(1, 300);
        const int path = k % 3;
        std::vector<int64_t> n(batch);
        std::vector<int32_t> M(batch), tile(batch);
        const bool one_m = (k % 4) == 0;
        const int32_t m0 = (int32_t)uniform(0, 256);
        for (int32_t s = 0; s < batch; ++s) {
            M[s] = one_m ? m0 : (int32_t)uniform(0, k % 5 == 0 ? 1024 : 300);
            n[s] = uniform(M[s] + 1 > 2 ? M[s] + 1 : 2, 70000);
            tile[s] = path == HOS_PATH_FP32 ? 4 : (int32_t)((int64_t[]){0, 2, 4}[uniform(0, 2)]);
        }
        uint32_t flags = (k % 2) ? HOS_NO_CENTER : 0u;
        if (one_m && (k % 8) == 0)
            flags |= HOS_PLAN_SEGMENTS;
        bool adj = false;
        if (one_m && m0 <= 320 && (k % 3) == 1) {
            flags |= HOS_PLAN_ADJOINT;
            adj = true;
        }
        size_t pb = 0, wb = 0;
        const int st = hos_batch_plan_size(batch, n.data(), M.data(), HOS_WIN_PARZEN, path, flags,
                                           (k % 2) ? tile.data() : nullptr, &pb, &wb);
        CHECK(st == HOS_OK);
        if (st != HOS_OK)
            continue;
        // the plan in a buffer of exactly pb bytes (8-byte aligned)
        std::vector<uint64_t> blob((pb + 7) / 8);
        CHECK(hos_batch_plan(batch, n.data(), M.data(), HOS_WIN_PARZEN, path, flags,
                             (k % 2) ? tile.data() : nullptr, blob.data(), pb) == HOS_OK);
        int64_t info[12];
        CHECK(hos_batch_plan_info(blob.data(), info, 12) == HOS_OK);
        std::vector<int64_t> ser(8 * (size_t)batch);
        CHECK(hos_batch_series(blob.data(), ser.data(), (int64_t)ser.size()) == HOS_OK);
        for (int cls = -1; cls <= 1; ++cls) {
            const int64_t ni = cls < 0 ? info[6] + info[7] : info[6 + cls];
            std::vector<int64_t> it(8 * (size_t)(ni > 0 ? ni : 1));
            CHECK(hos_batch_items(blob.data(), cls, it.data(), 8 * ni) == HOS_OK);
        }
        (void)adj;
    }
    // windows beyond the hexagon and bad sizes are refused
    int64_t n1 = 5000;
    int32_t m1 = 40;
    size_t pb, wb;
    CHECK(hos_batch_plan_size(1, &n1, &m1, HOS_WIN_NONE, 1, 0, nullptr, &pb, &wb) ==
          HOS_EUNSUPPORTED);
    m1 = 5000;
    CHECK(hos_batch_plan_size(1, &n1, &m1, HOS_WIN_PARZEN, 1, 0, nullptr, &pb, &wb) == HOS_EINVAL);
}

static void dbs_plans()
{
    const int32_t Ps[6] = {2, 3, 128, 1000, 4096, 65536};
    for (int k = 0; k < 24; ++k) {
        const int32_t P = Ps[k % 6];
        const int64_t n = P * uniform(1, 8) + uniform(0, 5);
        const int32_t M3 = (int32_t)uniform(1, P < 2048 ? P : 2048);
        int64_t info[16];
        hos_dbs_plan_info(n, P, M3, 0, 0, info, 16);
        size_t b = 0;
        hos_dbs_workspace(n, P, M3, &b);
    }
}

static void streamed_and_tune()
{
    size_t b = 0;
    CHECK(hos_bispectrum_streamed_workspace(1 << 26, 512, 1024, 1, HOS_F32, 1 << 22, &b) == HOS_OK);
    CHECK(hos_bispectrum_streamed_workspace(100000, 5, 16, 0, HOS_F64, 4096, &b) == HOS_OK);
    const int32_t Ms[4] = {32, 64, 128, 256};
    const int64_t edges[5] = {1024, 4096, 16384, 32768, 65537};
    for (int path = 0; path < 3; ++path)
        CHECK(hos_tune_workspace(path, Ms, 4, edges, 4, 16, &b) == HOS_OK);
}

static void validation()
{
    // rejected before any HIP call: fake, aligned device addresses
    char *fake = (char *)(uintptr_t)0x100000;
    CHECK(hos_bispectrum(fake, HOS_F32, 1, 0, 1, 8, 0, 0, (double *)fake, nullptr, fake, 1 << 20,
                         nullptr) == HOS_EINVAL);
    CHECK(hos_bispectrum(fake, HOS_F32, 4096, 64, 1, 128, 0, 0, (double *)fake, nullptr, fake, 16,
                         nullptr) == HOS_EWORKSPACE);
    CHECK(hos_bispectrum_noalloc(fake, HOS_F32, 1 << 22, 512, 1, 0, 1, 0, (double *)fake,
                                 nullptr, nullptr) == HOS_ESCRATCH);
    CHECK(hos_trispectrum(fake, HOS_F32, 4096, 20, HOS_WIN_NONE, 41, 0, 0, (double *)fake,
                          nullptr, fake, 1 << 30, nullptr) == HOS_EUNSUPPORTED);
    CHECK(hos_cumulant5(fake, HOS_F32, 4096, 8, HOS_WIN_PARZEN, 16, 0, 0, (double *)fake, nullptr,
                        fake, 16, nullptr) == HOS_EWORKSPACE);
    for (int s = -7; s <= 1; ++s)
        CHECK(hos_strerror(s) != nullptr);
}

int main()
{
    c3_plans();
    high_order_plans();
    batch_plans();
    dbs_plans();
    streamed_and_tune();
    validation();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host driver: ok\n");
    return 0;
}
