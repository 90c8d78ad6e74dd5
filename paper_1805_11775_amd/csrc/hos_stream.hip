// hos_stream.hip -- the bispectrum of a record held in host memory, streamed
// through a device workspace whose size depends on the piece length and M,
// not on n (the memory frugality of Section 3's window-sum theorems, applied
// to the indirect estimator).
//
// The record is read twice.  Pass one gives the whole record's FP64 mean
// and scale.  A record in pinned host memory that the device addresses at
// the same address (hipHostMalloc'd, or registered as mapped) is read in
// place by the moments kernels of the in-memory call, in one launch over
// the whole record, with no copies and no host calls per piece; any other
// record is copied piece by piece (P samples a piece) and the sum, minimum
// and maximum are accumulated in FP64, in piece order.  Pass two copies each piece together
// with the next M samples (its halo) and runs the single-series stages on
// it: the operands are rounded with the keys of their place in the record,
// the first factor x_i stops at the piece's end, so the contraction and the
// diagonal sums add exactly the terms with i in the piece; the piece's
// reduced table is added to a running FP64 table.  The sum over the pieces
// is the sum over the record, so the result is the whole record's c3 and B
// (up to the order of FP64 additions).
//
// Copies run on a copy stream of the library's own (one per device, made
// at first use, default priority) into two staging buffers taken in turn:
// the copy of the next piece overlaps the kernels of the current one.
// Events order the two streams both ways: a piece's kernels wait until its
// copy has landed, and a copy into a buffer waits until the kernels of the
// piece it held two steps earlier are done (and, for the first two copies,
// until the caller's stream has reached the call, which may still be using
// the workspace).
#include <mutex>
#include <string.h>

#include "hos_internal.h"

namespace hos {

namespace {

__global__ void __launch_bounds__(256)
k_table_add(double *__restrict__ acc, const double *__restrict__ add, int64_t count, int first)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count)
        return;
    acc[e] = first ? add[e] : acc[e] + add[e];
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// samples piece k reads: its own, then up to `halo` of the next pieces' (M,
// or 2M when the square's corners are computed)
int64_t piece_len(int64_t n, int64_t P, int64_t k) { return n - k * P < P ? n - k * P : P; }
int64_t piece_data(int64_t n, int64_t halo, int64_t P, int64_t k)
{
    const int64_t len = piece_len(n, P, k), rest = n - k * P;
    return rest < len + halo ? rest : len + halo;
}

struct StreamLayout {
    int64_t P, halo;          // piece length, halo samples
    size_t plan_bytes;        // largest single-series plan of a piece
    size_t off_acc, off_mom, off_x[2], total;
};

int stream_layout(int64_t n, int32_t M, int32_t nfft, int32_t path, int64_t P, int esize,
                  StreamLayout &L)
{
    memset(&L, 0, sizeof(L));
    L.P = P;
    L.halo = 2 * (int64_t)M;   // the layout covers the corners whatever the window
    // pieces k hold samples [kP, kP + len) and read data = min(len + halo,
    // n - kP) of them; every piece before the last two reads the same data
    // run as piece 0, so the plans of pieces 0, pieces-2 and pieces-1 bound
    // them all (a shorter halo only shrinks a plan)
    const int64_t pieces = (n + P - 1) / P;
    size_t mx = 0;
    int64_t data_max = 0;
    for (int64_t k : {(int64_t)0, pieces - 2, pieces - 1}) {
        if (k < 0)
            continue;
        const int64_t data = piece_data(n, L.halo, P, k);
        C3Plan p;
        make_c3_plan(data, M, path, nfft, p, true);
        if (p.total > mx)
            mx = p.total;
        if (data > data_max)
            data_max = data;
    }
    L.plan_bytes = al256(mx);
    size_t o = L.plan_bytes;
    L.off_acc = o;  o = al256(o + (size_t)(M + 1) * (M + 1) * sizeof(double));
    L.off_mom = o;  o = al256(o + 4 * sizeof(double));
    L.off_x[0] = o; o = al256(o + (size_t)data_max * esize);
    L.off_x[1] = o; o = al256(o + (size_t)data_max * esize);
    L.total = o;
    return HOS_OK;
}

constexpr int STREAM_MAX_DEVICES = 64;

// The copy stream of the current device, made once and kept until the
// process ends.
hipError_t copy_stream(hipStream_t &cs)
{
    static std::mutex mu;
    static hipStream_t streams[STREAM_MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= STREAM_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    cs = streams[dev];
    return hipSuccess;
}

// Staging of the record's pieces through the two buffers (see the top of
// the file).  put() copies bytes from the host into the next buffer and
// makes the caller's stream wait for it; done() marks the end of the
// kernels that read the buffer put() returned last.
struct Stager {
    hipStream_t s = nullptr, cs = nullptr;
    hipEvent_t start = nullptr, ready[2] = {}, freed[2] = {};
    char *buf[2] = {};
    int64_t step = 0;

    hipError_t init(hipStream_t stream, char *b0, char *b1)
    {
        s = stream;
        buf[0] = b0;
        buf[1] = b1;
        hipError_t e = copy_stream(cs);
        hipEvent_t *all[5] = {&start, &ready[0], &ready[1], &freed[0], &freed[1]};
        for (hipEvent_t *ev : all)
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(start, s);
        return e;
    }
    hipError_t put(const char *src, size_t bytes, char *&dst)
    {
        const int b = (int)(step & 1);
        hipError_t e = hipStreamWaitEvent(cs, step < 2 ? start : freed[b], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(buf[b], src, bytes, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess)
            e = hipEventRecord(ready[b], cs);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, ready[b], 0);
        dst = buf[b];
        return e;
    }
    hipError_t done()
    {
        return hipEventRecord(freed[(step++) & 1], s);
    }
    // Events still pending are released by the runtime once they complete;
    // the caller's stream has waited for every copy, so its completion
    // implies theirs.
    ~Stager()
    {
        hipEvent_t all[5] = {start, ready[0], ready[1], freed[0], freed[1]};
        for (hipEvent_t ev : all)
            if (ev)
                hipEventDestroy(ev);
    }
};

// True when the device can read [x, x + bytes) in place: pinned host memory
// mapped at the same address, the whole range inside one allocation.  A
// failed query (pageable memory) is cleared so that it does not surface as
// the error of a later launch.
bool device_visible(const void *x, size_t bytes)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, x) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeHost)
        return false;
    void *dp = nullptr;
    if (hipHostGetDevicePointer(&dp, const_cast<void *>(x), 0) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    hipDeviceptr_t start = nullptr;
    size_t size = 0;
    if (hipPointerGetAttribute(&start, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR,
                               (hipDeviceptr_t)x) != hipSuccess ||
        hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, (hipDeviceptr_t)x) !=
            hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t lo = (uintptr_t)start, p = (uintptr_t)x;
    return dp == x && start != nullptr && p >= lo && bytes <= size && p - lo <= size - bytes;
}

}  // namespace

}  // namespace hos

using namespace hos;

static bool st_aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr & (a - 1)) == 0; }

static int check_stream_args(int64_t n, int32_t M, int32_t window, int32_t nfft, int32_t path,
                             uint32_t flags, int64_t P, bool want_B)
{
    if (n < 2 || n > ((int64_t)1 << 40) || M < 0 || (int64_t)M >= n || M > 8192)
        return HOS_EINVAL;
    if (P < 4096 || P > ((int64_t)1 << 31) || P < M || P % 1024 != 0)
        return HOS_EINVAL;
    if (path != HOS_PATH_FP32 && path != HOS_PATH_SPLIT_FP16 && path != HOS_PATH_SPLIT_BF16)
        return HOS_EINVAL;
    if (window != HOS_WIN_NONE && window != HOS_WIN_PARZEN && window != HOS_WIN_PARZEN_SEPARABLE)
        return HOS_EINVAL;
    if (flags & ~(HOS_NO_CENTER | HOS_FULL_SQUARE))
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

extern "C" {

int hos_bispectrum_streamed_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path,
                                      int32_t dtype, int64_t piece, size_t *bytes)
{
    if (!bytes || (dtype != HOS_F32 && dtype != HOS_F64))
        return HOS_EINVAL;
    int st = check_stream_args(n, M, HOS_WIN_NONE, 0, path, 0, piece, false);
    if (st != HOS_OK)
        return st;
    if (nfft > 0 && !fft_size_ok(nfft))
        return HOS_EINVAL;
    StreamLayout L;
    stream_layout(n, M, nfft > 0 ? nfft : 0, path, piece, dtype == HOS_F64 ? 8 : 4, L);
    *bytes = L.total;
    return HOS_OK;
}

int hos_bispectrum_streamed(const void *x_host, int32_t dtype, int64_t n, int32_t M,
                            int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                            int64_t piece, double *c3, double *B, void *ws, size_t ws_bytes,
                            hipStream_t stream)
{
    if (!x_host || !ws || (!c3 && !B))
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!st_aligned(ws, 256) || (c3 && !st_aligned(c3, 8)) || (B && !st_aligned(B, 16)))
        return HOS_EINVAL;
    int st = check_stream_args(n, M, window, nfft, path, flags, piece, B != nullptr);
    if (st != HOS_OK)
        return st;
    const int esize = dtype == HOS_F64 ? 8 : 4;
    StreamLayout L;
    stream_layout(n, M, B ? nfft : 0, path, piece, esize, L);
    if (ws_bytes < L.total)
        return HOS_EWORKSPACE;
    st = device_ok_public();
    if (st != HOS_OK)
        return st;

    char *w = (char *)ws;
    double *acc = (double *)(w + L.off_acc);
    double *mom = (double *)(w + L.off_mom);
    const char *xh = (const char *)x_host;
    const int64_t pieces = (n + piece - 1) / piece;
    Stager stg;
    hipError_t e = stg.init(stream, w + L.off_x[0], w + L.off_x[1]);

    // pass one: the record's mean and scale into the stats every piece plan
    // reads (each plan puts its stats at offset 0 of the workspace; p0 is
    // the plan of a full piece with its halo, within the workspace layout)
    C3Plan p0;
    const bool corners = bispectrum_needs_corners(window, flags, B != nullptr);
    const int64_t halo = corners ? 2 * (int64_t)M : M;
    make_c3_plan(piece_data(n, halo, piece, 0), M, path, B ? nfft : 0, p0, corners);
    double *stats = (double *)(w + p0.off_stats);
    const bool direct = device_visible(x_host, (size_t)n * esize);
    char *xd = nullptr;
    if (direct) {   // in place, as the in-memory call does it
        if (e == hipSuccess)
            e = launch_moments(x_host, dtype, n, flags, p0, w, stream);
    } else {        // sum, minimum, maximum piece by piece
        for (int64_t k = 0; k < pieces && e == hipSuccess; ++k) {
            const int64_t g0 = k * piece, len = piece_len(n, piece, k);
            // a record of one piece is staged whole (it is its own halo)
            // and read again by pass two from the same buffer
            const int64_t cp = pieces == 1 ? n : len;
            e = stg.put(xh + g0 * esize, (size_t)cp * esize, xd);
            if (e == hipSuccess)
                e = launch_moments_piece(xd, dtype, len, k == 0, p0, w, mom, stream);
            if (e == hipSuccess && pieces > 1)
                e = stg.done();
        }
        if (e == hipSuccess)
            e = launch_moments_total(mom, n, flags, p0.scale_top, stats, stream);
    }
    // a one-piece record staged by pass one is already in its buffer
    const bool staged_whole = !direct && pieces == 1;

    // pass two: each piece with its halo through the single-series stages
    const int64_t ne = (int64_t)(M + 1) * (M + 1);
    for (int64_t k = 0; k < pieces && e == hipSuccess; ++k) {
        const int64_t g0 = k * piece, len = piece_len(n, piece, k);
        const int64_t data = piece_data(n, halo, piece, k);
        C3Plan p;
        make_c3_plan(data, M, path, B ? nfft : 0, p, corners);
        if (al256(p.total) > L.plan_bytes) {   // the layout bounds every piece's plan
            e = hipErrorInvalidValue;
            break;
        }
        if (!staged_whole)
            e = stg.put(xh + g0 * esize, (size_t)data * esize, xd);
        if (e == hipSuccess) e = launch_prep(xd, dtype, p, w, stream, g0, len);
        if (e == hipSuccess) e = launch_c3_contract(p, w, stream, 0);
        if (e == hipSuccess) e = launch_diag_dot(xd, dtype, p, w, stream, len);
        if (e == hipSuccess) e = launch_c3_reduce(p, w, stream, 0);
        if (e == hipSuccess && corners) e = launch_c3_contract(p, w, stream, 1);
        if (e == hipSuccess && corners) e = launch_c3_reduce(p, w, stream, 1);
        if (e == hipSuccess && pieces > 1) e = stg.done();
        if (e == hipSuccess) {
            k_table_add<<<(unsigned)((ne + 255) / 256), 256, 0, stream>>>(
                acc, (const double *)(w + p.off_cfull), ne, k == 0);
            e = hipGetLastError();
        }
    }
    // normalise by the whole record (stats[3] = n s^3), window, DFT
    if (e == hipSuccess) {
        double2 *tw = B ? (double2 *)(w + p0.off_twid) : nullptr;
        if (B)
            e = launch_twiddles(tw, nfft, stream);
        if (e == hipSuccess)
            e = launch_c3_finish_table(acc, stats, M, p0.amax, window, nfft, tw, c3,
                                       (flags & HOS_FULL_SQUARE) ? 2 * M : M, B, stream);
        if (e == hipSuccess && B)
            e = launch_fft_cols(B, nfft, tw, stream);
    }
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

}  // extern "C"
