// hos_api.hip -- C ABI entry points: validation, planning, launch order.
//
// Every argument is validated on the host before the first HIP call, so a
// rejected call leaves the device untouched.  The library keeps no state
// between calls except a per-device "is this a gfx950" flag.
#include <string.h>

#include <mutex>

#include "hos_internal.h"

namespace hos {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int make_c3_plan(int64_t n, int32_t M, int32_t path, int32_t nfft, C3Plan &p, bool corners,
                 bool full_grid)
{
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.M = M;
    p.path = path;
    p.scale_top = 7;
    p.amax = corners ? 2 * M : M;
    // Split paths: 4 column blocks per wave amortise the product-row split
    // (2-block tiles for small M); FP32 path: 128 x 128 tiles with a 2 x 2
    // block window per wave.
    p.NB = (M >= 96 || path == HOS_PATH_FP32) ? 4 : 2;
    p.TS = 32 * p.NB;
    p.NBR = (M + 31) / 32;
    p.nleft = 1 + M / 32;
    const int64_t KCX = c3_stage_len(path, p.NB);   // samples per chunk
    const int64_t C = (n + KCX - 1) / KCX;
    SkGeom &g = p.sk;
    g.TR = p.NBR > 0 ? (p.NBR + p.NB - 1) / p.NB : 0;
    // a tile's time is set by its busiest wave: a strip of NB blocks on every
    // tile (split paths); 4 blocks off and 3 on the diagonal (FP32 layout)
    g.cf = path == HOS_PATH_FP32 ? 4 : 1;
    g.cd = path == HOS_PATH_FP32 ? 3 : 1;
    g.C = C;
    g.ctot = g.TR > 0 ? sk_row_prefix(g, g.TR) * C : 0;
    int64_t G = g.ctot / g.cf;  // every workgroup's range holds >= 1 chunk start
    const int64_t gmax = p.NB == 4 ? SK_MAX_WG : 2 * SK_MAX_WG;  // 2-wave groups pair up
    if (G > gmax)
        G = gmax;
    if (G < 1)
        G = 1;
    g.G = (int32_t)G;
    p.smax = g.TR > 0 ? sk_max_segments(g) : 0;
    // the corner contraction reads its Hankel columns M + 1 samples further on
    const int64_t coff = p.amax > M ? (int64_t)M + 1 : 0;
    p.npad = ((C * KCX + (int64_t)g.TR * p.TS + coff + 64) + 63) / 64 * 64;
    // leftover diagonal sums: one pass over x in 1024-sample blocks
    // (k_diag_fused) when nleft <= 32, else nleft x 64 strided blocks
    if (p.nleft <= 32) {
        p.dot_blocks = (int32_t)((n + 1023) / 1024);
    } else {
        const int64_t db = n / 4096;
        p.dot_blocks = (int32_t)(db < 1 ? 1 : (db > 64 ? 64 : db));
    }

    size_t o = 0;
    p.off_stats = o;  o = align256(o + 64 * sizeof(double));
    p.off_mpart = o;  o = align256(o + MOM_BLOCKS * 3 * sizeof(double));
    p.off_xf = o;     o = align256(o + (size_t)p.npad * sizeof(float));
    p.off_win4 = o;   o = align256(o + (size_t)p.npad * 16);
    if (path != HOS_PATH_FP32) {
        p.off_win8h = o;  o = align256(o + (size_t)p.npad * 16);
        p.off_win8l = o;  o = align256(o + (size_t)p.npad * 16);
    }
    if (M > 0) {
        p.off_part = o;
        o = align256(o + (size_t)g.G * p.smax * tile_elems(p.NB) * sizeof(double));
        p.off_tfirst = o;
        o = align256(o + (size_t)g.G * sizeof(int64_t));
    }
    p.off_cfull = o;  o = align256(o + (size_t)(M + 1) * (M + 1) * sizeof(double));
    p.off_dpart = o;  o = align256(o + (size_t)p.nleft * p.dot_blocks * sizeof(double));
    if (nfft > 0) {
        p.off_twid = o;
        o = align256(o + (size_t)nfft * 2 * sizeof(double));
        if (full_grid) {
            p.off_bfull = o;
            o = align256(o + (size_t)nfft * nfft * 2 * sizeof(double));
        }
    }
    p.total = o;
    return HOS_OK;
}

int make_c4_plan(int64_t n, int32_t M, int32_t path, int32_t nfft, C4Plan &p, int ord)
{
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.M = M;
    p.path = path;
    p.ord = ord;
    // the split paths round the product rows to FP16: |x~ s| < 32 keeps a
    // product of three samples below 2^15, |x~ s| < 8 one of four
    p.scale_top = ord == 5 ? 3 : 5;
    p.P = ord == 5 ? (M + 1) * (M + 2) * (M + 3) / 6 : (M + 1) * (M + 2) / 2;
    p.RB = (p.P + 31) / 32;
    p.NCB = (M + 1 + 31) / 32;
    p.WX = c4_window_entries(M);
    p.C = (n + KC - 1) / KC;
    // about two workgroups per compute unit; every range holds >= 1 chunk
    const int64_t rbg = (p.RB + 3) / 4;
    int64_t S = (512 + rbg - 1) / rbg;
    if (S > p.C)
        S = p.C;
    if (S < 1)
        S = 1;
    const int64_t cps = (p.C + S - 1) / S;
    p.CPS = (int32_t)cps;
    p.S = (int32_t)((p.C + cps - 1) / cps);
    p.npad = ((p.C * KC + p.WX + 64) + 63) / 64 * 64;
    int64_t db = n / 4096;
    p.dot_blocks = (int32_t)(db < 1 ? 1 : (db > 64 ? 64 : db));
    const int64_t c3b = (n + C3D_BS - 1) / C3D_BS;
    p.c3_blocks = (int32_t)(c3b > C3D_MAX_WG ? C3D_MAX_WG : c3b);

    size_t o = 0;
    p.off_stats = o;  o = align256(o + 64 * sizeof(double));
    p.off_mpart = o;  o = align256(o + MOM_BLOCKS * 3 * sizeof(double));
    p.off_xf = o;     o = align256(o + (size_t)p.npad * sizeof(float));
    p.off_win4 = o;   o = align256(o + (size_t)p.npad * 16);
    if (path != HOS_PATH_FP32) {
        p.off_win8h = o;  o = align256(o + (size_t)p.npad * 16);
        p.off_win8l = o;  o = align256(o + (size_t)p.npad * 16);
    }
    p.off_part = o;
    o = align256(o + (size_t)p.S * p.RB * p.NCB * 1024 * sizeof(double));
    p.off_m4 = o;     o = align256(o + (size_t)p.P * (M + 1) * sizeof(double));
    p.off_c2part = o; o = align256(o + (size_t)(M + 1) * p.dot_blocks * sizeof(double));
    p.off_c2 = o;     o = align256(o + (size_t)(M + 1) * sizeof(double));
    if (ord == 5) {
        p.off_c3part = o;
        o = align256(o + (size_t)(M + 1) * (M + 2) / 2 * p.c3_blocks * sizeof(double));
        p.off_c3tab = o;
        o = align256(o + (size_t)(M + 1) * (M + 1) * sizeof(double));
    }
    if (nfft > 0) {
        p.off_twid = o;
        o = align256(o + (size_t)nfft * 2 * sizeof(double));
        // the cumulant cube the spectrum folds (used when the caller asks
        // for the spectrum alone)
        const size_t side = 2 * (size_t)M + 1;
        const size_t cube = ord == 5 ? side * side * side * side : side * side * side;
        p.off_cube = o;
        o = align256(o + cube * sizeof(double));
    }
    p.total = o;
    return HOS_OK;
}

static bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr & (a - 1)) == 0; }

// n is capped at 2^31 samples: the one-dimensional grids over the padded
// series (operand tables, diagonal sums) then stay far inside the 32-bit
// work-item range of a launch.
constexpr int64_t MAX_SERIES = (int64_t)1 << 31;

static int check_bispectrum_args(int64_t n, int32_t M, int32_t window, int32_t nfft,
                                 int32_t path, uint32_t flags, bool want_B,
                                 uint32_t allowed = HOS_NO_CENTER)
{
    if (n < 2 || n > MAX_SERIES)
        return HOS_EINVAL;
    if (M < 0 || (int64_t)M >= n || M > 8192)
        return HOS_EINVAL;
    if (path != HOS_PATH_FP32 && path != HOS_PATH_SPLIT_FP16 && path != HOS_PATH_SPLIT_BF16)
        return HOS_EINVAL;
    if (window != HOS_WIN_NONE && window != HOS_WIN_PARZEN && window != HOS_WIN_PARZEN_SEPARABLE)
        return HOS_EINVAL;
    if (flags & ~allowed)
        return HOS_EINVAL;
    if (want_B) {
        if (!fft_size_ok(nfft))
            return HOS_EINVAL;
        const int64_t need = window != HOS_WIN_NONE ? 2 * (int64_t)M : 2 * (int64_t)M + 1;
        if (nfft < need || nfft < 2)
            return HOS_EINVAL;
    } else if (nfft < 0) {
        return HOS_EINVAL;
    }
    return HOS_OK;
}

static int check_c5_args(int64_t n, int32_t M, int32_t window, int32_t nfft, int32_t path,
                         uint32_t flags, bool want_Q)
{
    if (M > C5_MAX_M)
        return HOS_EINVAL;
    if (want_Q && nfft > C5_MAX_NFFT)
        return HOS_EINVAL;
    return check_bispectrum_args(n, M, window, nfft, path, flags, want_Q);
}

// Windows the fourth- and fifth-order paths cover: their contractions fill
// the lags of span <= M only, where the Parzen product over every pairwise
// difference lives; the other windows need spans up to 2M.
static int check_high_order_window(int32_t window)
{
    return window == HOS_WIN_PARZEN ? HOS_OK : HOS_EUNSUPPORTED;
}

static int check_trispectrum_args(int64_t n, int32_t M, int32_t window, int32_t nfft,
                                  int32_t path, uint32_t flags, bool want_T)
{
    if (M > C4_MAX_M)
        return HOS_EINVAL;
    if (want_T && nfft > C4_MAX_NFFT)
        return HOS_EINVAL;
    return check_bispectrum_args(n, M, window, nfft, path, flags, want_T);
}

// Device gate: one check per device id, cached.
static int device_ok()
{
    static std::mutex mu;
    static int cache[64];
    static bool init = false;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return HOS_ENODEVICE;
    if (dev >= 64)
        return HOS_ENODEVICE;
    std::lock_guard<std::mutex> lk(mu);
    if (!init) {
        for (int &c : cache)
            c = 0;
        init = true;
    }
    if (cache[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return HOS_EDEVICE;
        cache[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    }
    return cache[dev] == 1 ? HOS_OK : HOS_ENODEVICE;
}

int device_ok_public() { return device_ok(); }

// The square's corners |w1 - w2| > M are computed when c3 is asked for them
// or when the window does not vanish there (everything but the Parzen
// product with d(w1 - w2), which is 0 from |w1 - w2| = M on).
bool bispectrum_needs_corners(int32_t window, uint32_t flags, bool want_B)
{
    return (flags & HOS_FULL_SQUARE) || (want_B && window != HOS_WIN_PARZEN);
}

// Host-side validation of a hos_bispectrum call (everything but the
// workspace) and its plan; no HIP call.
int bispectrum_check(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                          int32_t nfft, int32_t path, uint32_t flags, const double *c3,
                          const double *B, C3Plan &p)
{
    if (!x || (!c3 && !B))
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!aligned(x, dtype == HOS_F64 ? 8 : 4))
        return HOS_EINVAL;
    if ((c3 && !aligned(c3, 8)) || (B && !aligned(B, 16)))
        return HOS_EINVAL;
    int st = check_bispectrum_args(n, M, window, B ? nfft : 0, path, flags, B != nullptr,
                                   HOS_NO_CENTER | HOS_FULL_SQUARE | HOS_PD_ONLY);
    if (st != HOS_OK)
        return st;
    make_c3_plan(n, M, path, B ? nfft : 0, p, bispectrum_needs_corners(window, flags, B != nullptr),
                 B && (flags & HOS_PD_ONLY));
    return HOS_OK;
}

// Shared body of hos_bispectrum, hos_bispectrum_timed and
// hos_bispectrum_noalloc: validation, plan, and the launch sequence.  `ev`
// (8 events or NULL) brackets the stages.
int bispectrum_run(const void *x, int32_t dtype, int64_t n, int32_t M,
                           int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                           double *c3, double *B, void *ws, size_t ws_bytes,
                           hipStream_t stream, hipEvent_t *ev)
{
    if (!ws || !aligned(ws, 256))
        return HOS_EINVAL;
    C3Plan p;
    int st = bispectrum_check(x, dtype, n, M, window, nfft, path, flags, c3, B, p);
    if (st != HOS_OK)
        return st;
    if (ws_bytes < p.total)
        return HOS_EWORKSPACE;
    st = device_ok();
    if (st != HOS_OK)
        return st;

    char *w = (char *)ws;
    auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], stream) : hipSuccess; };
    double2 *tw = B ? (double2 *)(w + p.off_twid) : nullptr;
    const bool pd_only = B && (flags & HOS_PD_ONLY);
    // the N x N grid: the output itself, or staged in the workspace and then
    // reduced to its principal domain
    double *grid = pd_only ? (double *)(w + p.off_bfull) : B;
    const int c3_amax = (flags & HOS_FULL_SQUARE) ? 2 * M : M;
    hipError_t e = mark(0);
    if (e == hipSuccess) e = launch_moments(x, dtype, n, flags, p, w, stream);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess) e = launch_prep(x, dtype, p, w, stream);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = launch_c3_contract(p, w, stream, 0);
    if (e == hipSuccess) e = mark(3);
    if (e == hipSuccess) e = launch_diag_dot(x, dtype, p, w, stream);
    if (e == hipSuccess) e = mark(4);
    if (e == hipSuccess) e = launch_c3_reduce(p, w, stream, 0);
    // the square's corners: the same contraction with the Hankel columns
    // shifted by M + 1 samples, on the partial-sum region just reduced
    if (e == hipSuccess && p.amax > M) e = launch_c3_contract(p, w, stream, 1);
    if (e == hipSuccess && p.amax > M) e = launch_c3_reduce(p, w, stream, 1);
    if (e == hipSuccess) e = mark(5);
    if (e == hipSuccess && B) e = launch_twiddles(tw, nfft, stream);
    if (e == hipSuccess) e = launch_c3_finish(p, window, nfft, c3, c3_amax, grid, w, stream);
    if (e == hipSuccess) e = mark(6);
    if (e == hipSuccess && B) e = launch_fft_cols(grid, nfft, tw, stream);
    if (e == hipSuccess && pd_only) e = launch_pd_gather(grid, nfft, B, stream);
    if (e == hipSuccess) e = mark(7);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

}  // namespace hos

using namespace hos;

extern "C" {

const char *hos_strerror(int status)
{
    switch (status) {
    case HOS_OK: return "success";
    case HOS_EINVAL: return "invalid argument";
    case HOS_EWORKSPACE: return "workspace too small";
    case HOS_EDEVICE: return "HIP device error";
    case HOS_ENODEVICE: return "no gfx950 device available";
    case HOS_EUNSUPPORTED: return "unsupported request";
    case HOS_ESCRATCH: return "request exceeds the fixed scratch of the non-allocating entry point";
    default: return "unknown status";
    }
}

int hos_version(void) { return HOS_VERSION; }

int hos_device_check(void)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return HOS_ENODEVICE;
    return device_ok();
}

int hos_bispectrum_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path, uint32_t flags,
                             size_t *bytes)
{
    if (!bytes)
        return HOS_EINVAL;
    const int win = HOS_WIN_NONE;
    int st = check_bispectrum_args(n, M, win, nfft > 0 ? nfft : 0, path, flags, false,
                                   HOS_NO_CENTER | HOS_FULL_SQUARE | HOS_PD_ONLY);
    if (st != HOS_OK)
        return st;
    if (nfft > 0 && !fft_size_ok(nfft))
        return HOS_EINVAL;
    // every layout has room for the corners (the windows that are nonzero
    // there need them whatever the flags say); they cost M + 1 samples of
    // operand padding, the table keeps them in its upper triangle
    C3Plan p;
    make_c3_plan(n, M, path, nfft, p, true, nfft > 0 && (flags & HOS_PD_ONLY));
    *bytes = p.total;
    return HOS_OK;
}

int hos_bispectrum(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                   int32_t nfft, int32_t path, uint32_t flags, double *c3, double *B,
                   void *ws, size_t ws_bytes, hipStream_t stream)
{
    return bispectrum_run(x, dtype, n, M, window, nfft, path, flags, c3, B, ws, ws_bytes,
                           stream, nullptr);
}

int hos_bispectrum_timed(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                         int32_t nfft, int32_t path, uint32_t flags, double *c3, double *B,
                         void *ws, size_t ws_bytes, hipStream_t stream, float *stage_ms)
{
    if (!stage_ms)
        return HOS_EINVAL;
    hipEvent_t ev[8];
    int made = 0;
    for (; made < 8; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess)
            break;
    int st = made == 8 ? bispectrum_run(x, dtype, n, M, window, nfft, path, flags, c3, B,
                                         ws, ws_bytes, stream, ev)
                       : HOS_EDEVICE;
    if (st == HOS_OK) {
        if (hipEventSynchronize(ev[7]) != hipSuccess) {
            st = HOS_EDEVICE;
        } else {
            for (int k = 0; k < 7; ++k)
                if (hipEventElapsedTime(&stage_ms[k], ev[k], ev[k + 1]) != hipSuccess)
                    st = HOS_EDEVICE;
            if (hipEventElapsedTime(&stage_ms[7], ev[0], ev[7]) != hipSuccess)
                st = HOS_EDEVICE;
        }
    }
    for (int k = 0; k < made; ++k)
        hipEventDestroy(ev[k]);
    return st;
}

int hos_trispectrum_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path,
                              uint32_t flags, size_t *bytes)
{
    if (!bytes)
        return HOS_EINVAL;
    int st = check_trispectrum_args(n, M, HOS_WIN_NONE, nfft > 0 ? nfft : 0, path, flags,
                                    false);
    if (st != HOS_OK)
        return st;
    if (nfft > 0 && (!fft_size_ok(nfft) || nfft > C4_MAX_NFFT))
        return HOS_EINVAL;
    C4Plan p;
    make_c4_plan(n, M, path, nfft, p, 4);
    *bytes = p.total;
    return HOS_OK;
}

static int trispectrum_impl(const void *x, int32_t dtype, int64_t n, int32_t M,
                            int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                            double *c4, double *T, void *ws, size_t ws_bytes,
                            hipStream_t stream, hipEvent_t *ev)
{
    if (!x || !ws || (!c4 && !T))
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!aligned(x, dtype == HOS_F64 ? 8 : 4) || !aligned(ws, 256))
        return HOS_EINVAL;
    if ((c4 && !aligned(c4, 8)) || (T && !aligned(T, 16)))
        return HOS_EINVAL;
    int st = check_trispectrum_args(n, M, window, T ? nfft : 0, path, flags, T != nullptr);
    if (st == HOS_OK)
        st = check_high_order_window(window);
    if (st != HOS_OK)
        return st;
    C4Plan p;
    make_c4_plan(n, M, path, T ? nfft : 0, p, 4);
    if (ws_bytes < p.total)
        return HOS_EWORKSPACE;
    st = device_ok();
    if (st != HOS_OK)
        return st;

    char *w = (char *)ws;
    auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], stream) : hipSuccess; };
    double2 *tw = T ? (double2 *)(w + p.off_twid) : nullptr;
    hipError_t e = mark(0);
    if (e == hipSuccess) e = launch_moments(x, dtype, n, flags, p, w, stream);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess) e = launch_prep(x, dtype, p, w, stream);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = launch_c4_contract(p, w, stream);
    if (e == hipSuccess) e = mark(3);
    if (e == hipSuccess) e = launch_c4_reduce(x, dtype, p, w, stream);
    if (e == hipSuccess) e = mark(4);
    if (e == hipSuccess && T) e = launch_twiddles(tw, nfft, stream);
    if (e == hipSuccess) e = launch_c4_finish(p, window, nfft, c4, T, w, stream);
    if (e == hipSuccess) e = mark(5);
    if (e == hipSuccess && T) e = launch_fft3_tail(T, nfft, tw, stream);
    if (e == hipSuccess) e = mark(6);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

int hos_trispectrum(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                    int32_t nfft, int32_t path, uint32_t flags, double *c4, double *T,
                    void *ws, size_t ws_bytes, hipStream_t stream)
{
    return trispectrum_impl(x, dtype, n, M, window, nfft, path, flags, c4, T, ws, ws_bytes,
                            stream, nullptr);
}

int hos_trispectrum_timed(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                          int32_t nfft, int32_t path, uint32_t flags, double *c4, double *T,
                          void *ws, size_t ws_bytes, hipStream_t stream, float *stage_ms)
{
    if (!stage_ms)
        return HOS_EINVAL;
    hipEvent_t ev[7];
    int made = 0;
    for (; made < 7; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess)
            break;
    int st = made == 7 ? trispectrum_impl(x, dtype, n, M, window, nfft, path, flags, c4, T,
                                          ws, ws_bytes, stream, ev)
                       : HOS_EDEVICE;
    if (st == HOS_OK) {
        if (hipEventSynchronize(ev[6]) != hipSuccess) {
            st = HOS_EDEVICE;
        } else {
            for (int k = 0; k < 6; ++k)
                if (hipEventElapsedTime(&stage_ms[k], ev[k], ev[k + 1]) != hipSuccess)
                    st = HOS_EDEVICE;
            if (hipEventElapsedTime(&stage_ms[6], ev[0], ev[6]) != hipSuccess)
                st = HOS_EDEVICE;
        }
    }
    for (int k = 0; k < made; ++k)
        hipEventDestroy(ev[k]);
    return st;
}

// Host-only plan of the fourth-order contraction:
// info[0..7] = P, RB, NCB, WX, S, CPS, C, workspace bytes.
// Order five: the same stages as the trispectrum with lag-triple rows, the
// third-order corrections, and the 4-D fold and DFT.
static int cumulant5_impl(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                          int32_t nfft, int32_t path, uint32_t flags, double *c5, double *Q,
                          void *ws, size_t ws_bytes, hipStream_t stream, hipEvent_t *ev)
{
    if (!x || !ws || (!c5 && !Q))
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!aligned(x, dtype == HOS_F64 ? 8 : 4) || !aligned(ws, 256))
        return HOS_EINVAL;
    if ((c5 && !aligned(c5, 8)) || (Q && !aligned(Q, 16)))
        return HOS_EINVAL;
    int st = check_c5_args(n, M, window, Q ? nfft : 0, path, flags, Q != nullptr);
    if (st == HOS_OK)
        st = check_high_order_window(window);
    if (st != HOS_OK)
        return st;
    C4Plan p;
    make_c4_plan(n, M, path, Q ? nfft : 0, p, 5);
    if (ws_bytes < p.total)
        return HOS_EWORKSPACE;
    st = device_ok();
    if (st != HOS_OK)
        return st;
    char *w = (char *)ws;
    auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], stream) : hipSuccess; };
    double2 *tw = Q ? (double2 *)(w + p.off_twid) : nullptr;
    hipError_t e = mark(0);
    if (e == hipSuccess) e = launch_moments(x, dtype, n, flags, p, w, stream);
    if (e == hipSuccess) e = launch_prep(x, dtype, p, w, stream);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess) e = launch_c4_contract(p, w, stream);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = launch_c4_reduce(x, dtype, p, w, stream);
    if (e == hipSuccess && Q) e = launch_twiddles(tw, nfft, stream);
    if (e == hipSuccess) e = launch_c5_finish(p, window, nfft, c5, Q, w, stream);
    if (e == hipSuccess) e = mark(3);
    if (e == hipSuccess && Q) e = launch_fft4_tail(Q, nfft, tw, stream);
    if (e == hipSuccess) e = mark(4);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

int hos_cumulant5_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path, uint32_t flags,
                            size_t *bytes)
{
    if (!bytes)
        return HOS_EINVAL;
    int st = check_c5_args(n, M, HOS_WIN_NONE, nfft > 0 ? nfft : 0, path, flags, false);
    if (st != HOS_OK)
        return st;
    if (nfft > 0 && (!fft_size_ok(nfft) || nfft > C5_MAX_NFFT))
        return HOS_EINVAL;
    C4Plan p;
    make_c4_plan(n, M, path, nfft, p, 5);
    *bytes = p.total;
    return HOS_OK;
}

int hos_cumulant5(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                  int32_t nfft, int32_t path, uint32_t flags, double *c5, double *Q, void *ws,
                  size_t ws_bytes, hipStream_t stream)
{
    return cumulant5_impl(x, dtype, n, M, window, nfft, path, flags, c5, Q, ws, ws_bytes,
                          stream, nullptr);
}

int hos_cumulant5_timed(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                        int32_t nfft, int32_t path, uint32_t flags, double *c5, double *Q,
                        void *ws, size_t ws_bytes, hipStream_t stream, float *stage_ms)
{
    if (!stage_ms)
        return HOS_EINVAL;
    hipEvent_t ev[5];
    int made = 0;
    for (; made < 5; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess)
            break;
    int st = made == 5 ? cumulant5_impl(x, dtype, n, M, window, nfft, path, flags, c5, Q, ws,
                                        ws_bytes, stream, ev)
                       : HOS_EDEVICE;
    if (st == HOS_OK) {
        if (hipEventSynchronize(ev[4]) != hipSuccess) {
            st = HOS_EDEVICE;
        } else {
            for (int k = 0; k < 4; ++k)
                if (hipEventElapsedTime(&stage_ms[k], ev[k], ev[k + 1]) != hipSuccess)
                    st = HOS_EDEVICE;
            if (hipEventElapsedTime(&stage_ms[4], ev[0], ev[4]) != hipSuccess)
                st = HOS_EDEVICE;
        }
    }
    for (int k = 0; k < made; ++k)
        hipEventDestroy(ev[k]);
    return st;
}

static int moment_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo,
                            int ord)
{
    if (!info || ninfo < 8)
        return HOS_EINVAL;
    int st = ord == 5 ? check_c5_args(n, M, HOS_WIN_NONE, 0, path, 0, false)
                      : check_trispectrum_args(n, M, HOS_WIN_NONE, 0, path, 0, false);
    if (st != HOS_OK)
        return st;
    C4Plan p;
    make_c4_plan(n, M, path, 0, p, ord);
    info[0] = p.P;
    info[1] = p.RB;
    info[2] = p.NCB;
    info[3] = p.WX;
    info[4] = p.S;
    info[5] = p.CPS;
    info[6] = p.C;
    info[7] = (int64_t)p.total;
    return HOS_OK;
}

int hos_c4_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo)
{
    return moment_plan_info(n, M, path, info, ninfo, 4);
}

int hos_c5_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo)
{
    return moment_plan_info(n, M, path, info, ninfo, 5);
}

// Host-only introspection of the contraction schedule (no HIP call):
// info[0..9] = G, smax, TR, C, NB, NBR, nleft, npad, ctot, workspace bytes.
int hos_c3_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo)
{
    if (!info || ninfo < 10)
        return HOS_EINVAL;
    int st = check_bispectrum_args(n, M, HOS_WIN_NONE, 0, path, 0, false);
    if (st != HOS_OK)
        return st;
    C3Plan p;
    make_c3_plan(n, M, path, 0, p);
    info[0] = p.sk.G;
    info[1] = p.smax;
    info[2] = p.sk.TR;
    info[3] = p.sk.C;
    info[4] = p.NB;
    info[5] = p.NBR;
    info[6] = p.nleft;
    info[7] = p.npad;
    info[8] = p.sk.ctot;
    info[9] = (int64_t)p.total;
    return HOS_OK;
}

// Host-only replay of the contraction's work split: for every (tile, chunk)
// in schedule order, owner[k] receives the workgroup that processes it, as
// the kernel's own iteration finds it, and slot[k] the partial slot it
// writes; the reduce side's lookup of the same pair is returned in
// rslot[k].  Used to test the split without a GPU.
int hos_c3_schedule(int64_t n, int32_t M, int32_t path, int64_t *owner, int64_t *slot,
                    int64_t *rslot, int64_t cap)
{
    if (!owner || !slot || !rslot)
        return HOS_EINVAL;
    int st = check_bispectrum_args(n, M, HOS_WIN_NONE, 0, path, 0, false);
    if (st != HOS_OK)
        return st;
    C3Plan p;
    make_c3_plan(n, M, path, 0, p);
    const SkGeom &g = p.sk;
    const int64_t ntiles = (int64_t)g.TR * (g.TR + 1) / 2;
    if (cap < ntiles * g.C)
        return HOS_EINVAL;
    for (int64_t k = 0; k < ntiles * g.C; ++k)
        owner[k] = slot[k] = rslot[k] = -1;
    // kernel side
    for (int64_t w = 0; w < g.G; ++w) {
        const int64_t S0 = sk_wg_start(g, w), S1 = sk_wg_start(g, w + 1);
        SkPos q;
        if (!sk_first_chunk(g, S0, q) || sk_chunk_start(g, q.R, q.Cc, q.c) >= S1)
            continue;
        const int64_t tfirst = sk_tile_index(q.R, q.Cc);
        for (;;) {
            const int64_t t = sk_tile_index(q.R, q.Cc);
            const int64_t k = t * g.C + q.c;
            if (owner[k] != -1)
                owner[k] = -2;  // processed twice
            else
                owner[k] = w;
            slot[k] = w * p.smax + (t - tfirst);
            if (t - tfirst >= p.smax)
                slot[k] = -3;
            SkPos nq = q;
            if (!(sk_next(g, nq) && sk_chunk_start(g, nq.R, nq.Cc, nq.c) < S1))
                break;
            q = nq;
        }
    }
    // reduce side: for each tile, the workgroups it sums and their slots
    for (int R = 0; R < g.TR; ++R)
        for (int Cc = 0; Cc <= R; ++Cc) {
            const int64_t t = sk_tile_index(R, Cc);
            const int64_t w_lo = sk_owner(g, sk_chunk_start(g, R, Cc, 0));
            const int64_t w_hi = sk_owner(g, sk_chunk_start(g, R, Cc, g.C - 1));
            for (int64_t c = 0; c < g.C; ++c) {
                const int64_t w = sk_owner(g, sk_chunk_start(g, R, Cc, c));
                SkPos p0;
                sk_first_chunk(g, sk_wg_start(g, w), p0);
                int64_t s = w * p.smax + (t - sk_tile_index(p0.R, p0.Cc));
                if (w < w_lo || w > w_hi)
                    s = -4;
                rslot[t * g.C + c] = s;
            }
        }
    return HOS_OK;
}

}  // extern "C"
