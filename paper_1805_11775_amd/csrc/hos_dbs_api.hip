// hos_dbs_api.hip -- C ABI of the direct method (Algorithm DBS): argument
// validation, the launch plan, and the entry points.  As for the other
// entry points, every argument is checked on the host before the first HIP
// call.
#include <string.h>

#include "hos_internal.h"

namespace hos {

static size_t dbs_align(size_t v) { return (v + 255) & ~(size_t)255; }

static bool smooth235(int v)
{
    if (v < 2)
        return false;
    for (int r : {2, 3, 5})
        while (v % r == 0)
            v /= r;
    return v == 1;
}

static int check_dbs_args(int64_t n, int32_t P, int32_t M3, uint32_t flags)
{
    if (P < 2 || P > DBS_MAX_P || !smooth235(P))
        return HOS_EINVAL;
    if (n < P || n > ((int64_t)1 << 40))
        return HOS_EINVAL;
    if (M3 < 1 || M3 > P || M3 > DBS_MAX_M3)
        return HOS_EINVAL;
    if (flags & ~HOS_NO_CENTER)
        return HOS_EINVAL;
    return HOS_OK;
}

static int64_t pd_points(int H)
{
    int64_t s = 0;
    for (int r = 0; r <= H; ++r)
        s += (r < H - r ? r : H - r) + 1;
    return s;
}

int make_dbs_plan(int64_t n, int32_t P, int32_t M3, int32_t seg_rows, int32_t strip_w,
                  DbsPlan &p)
{
    memset(&p, 0, sizeof(p));
    DbsGeom &g = p.g;
    p.n = n;
    p.K = n / P;
    p.mode = p.K == 1 ? 0 : 1;
    g.P = P;
    g.M3 = M3;
    g.lo = M3 / 2;
    g.hi = M3 - 1 - g.lo;
    g.H = (P - 1) / 2;
    const int Hc = g.H / 2;                  // largest principal-domain column
    // part DFT: one LDS pass, or P1 x P2 with both factors as close as possible
    if (P <= DBS_LDS_FFT) {
        p.P1 = P;
        p.P2 = 1;
    } else {
        int best = 0;
        for (int d = 2; d <= DBS_LDS_FFT; ++d)
            if (P % d == 0 && P / d <= DBS_LDS_FFT) {
                const int q = P / d;
                if (!best || (d > q ? d - q : q - d) < (best > P / best ? best - P / best
                                                                        : P / best - best))
                    best = d;
            }
        p.P1 = best;
        p.P2 = P / best;
    }
    // strip width: W widened columns (4 per thread) hold the box's M3 - 1
    // extra columns and TW = W - M3 + 1 outputs; the widest of 512, 1024,
    // 2048 that the grid's columns fill (wider strips repeat less of the
    // box's overlap and run as fewer, longer row steps)
    g.W = 2048;
    if (Hc + M3 <= 1024)
        g.W = 1024;
    if (Hc + M3 <= 512)
        g.W = 512;
    if (strip_w > 0)
        g.W = strip_w;
    g.CPT = 4;
    g.TW = g.W - M3 + 1;
    g.NS = (Hc + 1 + g.TW - 1) / g.TW;
    g.rows = 0;
    for (int s = 0; s < g.NS; ++s)
        g.rows += (int64_t)g.H - 2 * (int64_t)s * g.TW + 1;
    // the strips' rows laid end to end and cut into equal runs, one per
    // workgroup, as many as fit on the chip at once (a run may cross into
    // the next strip; each strip part restarts its box)
    const int per_cu = g.W == 2048 ? 1 : (g.W == 1024 ? 2 : 4);
    const int64_t target = (int64_t)DBS_CUS * per_cu;
    int64_t R = seg_rows > 0 ? seg_rows : (g.rows + target - 1) / target;
    if (seg_rows <= 0 && R < 16)
        R = 16;
    g.R = (int32_t)R;
    g.NSEG = (int32_t)((g.rows + R - 1) / R);
    g.SC = (g.NS - 1) * g.TW + g.W;
    g.norm = 1.0 / ((double)p.K * (double)P * (double)M3 * (double)M3);
    p.SR = g.H + M3;
    p.npd = pd_points(g.H);
    if (p.mode == 1) {
        const int64_t tiles = (int64_t)((g.SC + 63) / 64) * ((p.SR + 63) / 64);
        int64_t G = (2048 + tiles - 1) / tiles;
        const int64_t gmax = p.K < 64 ? p.K : 64;
        if (G > gmax)
            G = gmax;
        if (G < 1)
            G = 1;
        const int64_t Kg = (p.K + G - 1) / G;
        p.Kg = (int32_t)Kg;
        p.G = (int32_t)((p.K + Kg - 1) / Kg);
    }
    const int bpp = (P + 2047) / 2048;
    size_t o = 0;
    p.off_mean = o;  o = dbs_align(o + (size_t)p.K * bpp * sizeof(double));
    p.off_F = o;     o = dbs_align(o + (size_t)p.K * P * 16);
    if (p.P2 > 1) {
        p.off_T = o;   o = dbs_align(o + (size_t)p.K * P * 16);
        p.off_tw1 = o; o = dbs_align(o + (size_t)p.P1 * 16);
        p.off_tw2 = o; o = dbs_align(o + (size_t)p.P2 * 16);
    }
    p.off_tw = o;    o = dbs_align(o + (size_t)P * 16);
    if (p.mode == 1) {
        p.off_S = o;
        o = dbs_align(o + (size_t)p.G * p.SR * g.SC * 16);
    }
    p.total = o;
    return HOS_OK;
}

static bool dbs_aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr & (a - 1)) == 0; }

// Tuning arguments of the timed entry point: rows per smoothing workgroup
// (>= 0) and widened strip width (0, or 512 / 1024 / 2048 and >= M3).
static bool tune_ok(int32_t seg_rows, int32_t strip_w, int32_t M3)
{
    if (seg_rows < 0)
        return false;
    if (strip_w == 0)
        return true;
    return (strip_w == 512 || strip_w == 1024 || strip_w == 2048) && strip_w >= M3;
}

static int dbs_impl(const void *x, int32_t dtype, int64_t n, int32_t P, int32_t M3,
                    uint32_t flags, double *B_pd, void *ws, size_t ws_bytes, hipStream_t stream,
                    int32_t seg_rows, int32_t strip_w, hipEvent_t *ev)
{
    if (!x || !B_pd || !ws)
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!dbs_aligned(x, dtype == HOS_F64 ? 8 : 4) || !dbs_aligned(B_pd, 16) ||
        !dbs_aligned(ws, 256))
        return HOS_EINVAL;
    int st = check_dbs_args(n, P, M3, flags);
    if (st != HOS_OK)
        return st;
    if (!tune_ok(seg_rows, strip_w, M3))
        return HOS_EINVAL;
    DbsPlan p;
    make_dbs_plan(n, P, M3, seg_rows, strip_w, p);
    if (ws_bytes < p.total)
        return HOS_EWORKSPACE;
    st = device_ok_public();
    if (st != HOS_OK)
        return st;
    return launch_dbs(x, dtype, flags, p, B_pd, (char *)ws, stream, ev) == hipSuccess
               ? HOS_OK
               : HOS_EDEVICE;
}

}  // namespace hos

using namespace hos;

extern "C" {

int hos_dbs_workspace(int64_t n, int32_t P, int32_t M3, size_t *bytes)
{
    if (!bytes)
        return HOS_EINVAL;
    int st = check_dbs_args(n, P, M3, 0);
    if (st != HOS_OK)
        return st;
    DbsPlan p;
    make_dbs_plan(n, P, M3, 0, 0, p);
    *bytes = p.total;
    return HOS_OK;
}

int hos_dbs(const void *x, int32_t dtype, int64_t n, int32_t P, int32_t M3, uint32_t flags,
            double *B_pd, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return dbs_impl(x, dtype, n, P, M3, flags, B_pd, ws, ws_bytes, stream, 0, 0, nullptr);
}

int hos_dbs_timed(const void *x, int32_t dtype, int64_t n, int32_t P, int32_t M3,
                  uint32_t flags, double *B_pd, void *ws, size_t ws_bytes, hipStream_t stream,
                  int32_t seg_rows, int32_t strip_w, float *stage_ms)
{
    if (!stage_ms)
        return HOS_EINVAL;
    // the checks of dbs_impl, before any HIP call (events included)
    if (!x || !B_pd || !ws || (dtype != HOS_F32 && dtype != HOS_F64))
        return HOS_EINVAL;
    int vst = check_dbs_args(n, P, M3, flags);
    if (vst != HOS_OK)
        return vst;
    if (!tune_ok(seg_rows, strip_w, M3))
        return HOS_EINVAL;
    hipEvent_t ev[4];
    int made = 0;
    for (; made < 4; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess)
            break;
    int st = made == 4 ? dbs_impl(x, dtype, n, P, M3, flags, B_pd, ws, ws_bytes, stream,
                                  seg_rows, strip_w, ev)
                       : HOS_EDEVICE;
    if (st == HOS_OK) {
        if (hipEventSynchronize(ev[3]) != hipSuccess) {
            st = HOS_EDEVICE;
        } else {
            for (int k = 0; k < 3; ++k)
                if (hipEventElapsedTime(&stage_ms[k], ev[k], ev[k + 1]) != hipSuccess)
                    st = HOS_EDEVICE;
            if (hipEventElapsedTime(&stage_ms[3], ev[0], ev[3]) != hipSuccess)
                st = HOS_EDEVICE;
        }
    }
    for (int k = 0; k < made; ++k)
        hipEventDestroy(ev[k]);
    return st;
}

int hos_dbs_plan_info(int64_t n, int32_t P, int32_t M3, int32_t seg_rows, int32_t strip_w,
                      int64_t *info, int32_t ninfo)
{
    if (!info || ninfo < 16)
        return HOS_EINVAL;
    int st = check_dbs_args(n, P, M3, 0);
    if (st != HOS_OK)
        return st;
    if (!tune_ok(seg_rows, strip_w, M3))
        return HOS_EINVAL;
    DbsPlan p;
    make_dbs_plan(n, P, M3, seg_rows, strip_w, p);
    const int64_t v[16] = {p.K, p.mode, p.P1, p.P2, p.g.W, p.g.TW, p.g.NS, p.g.R,
                           p.g.NSEG, p.SR, p.g.SC, p.G, p.Kg, p.npd, (int64_t)p.total,
                           p.g.rows};
    for (int k = 0; k < 16; ++k)
        info[k] = v[k];
    return HOS_OK;
}

}  // extern "C"
