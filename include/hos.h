/*
 * hos.h -- C ABI of the MI355X (gfx950) higher-order-spectra library.
 *
 * The library estimates the smoothed sample bispectrum and trispectrum of a
 * finite real series (arXiv:1805.11775, Section 1 "Problem Statement": from
 * X(1..n), compute smoothed sample bispectrum and trispectrum that are
 * consistent estimates of the true higher-order spectra).  It follows the
 * indirect route the paper names in Section 1 ("Direct Method for HOS"):
 * sample cumulant over all lags |w| <= M, lag window, then the DFT.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Memory.    Every array argument is DEVICE memory owned by the caller unless
 *            the parameter says "host".  The library allocates nothing on the
 *            call path; scratch space is the caller's workspace `ws`
 *            (query its size first, 256-byte aligned).  No pointer is kept
 *            after the call returns.
 * Streams.   All work is enqueued on `stream` (NULL = the default stream) and
 *            the call returns without waiting for it.  Results are ready
 *            when the stream is synchronised.  hos_bispectrum and
 *            hos_trispectrum enqueue kernels only (no allocation, copy,
 *            memset or host wait), so a call can be captured into a HIP
 *            graph and replayed; the *_timed variants, the streamed entry
 *            point and hos_tune wait on the host and cannot be captured.
 * Errors.    Every function returns an hos_status code; no exception or
 *            abort crosses the ABI.  Arguments are validated on the host,
 *            before any HIP call, so a rejected call touches no device state.
 *            HOS_EDEVICE reports a HIP launch failure.
 * Estimator. x~_t = x_t - mean(x) (FP64 mean; skipped with HOS_NO_CENTER),
 *            c3(w1,w2) = (1/n) sum_t x~_t x~_{t+w1} x~_{t+w2} with the sum
 *            over the t where every index lies in [0,n) (zero padding).
 *            Internally x~ is multiplied by an exact power of two chosen
 *            from max|x~| and divided out again, so results do not depend
 *            on the input scale.
 *            c4(t1,t2,t3) = m4(t1,t2,t3) - c2(t1) c2(t3-t2) - c2(t2) c2(t3-t1)
 *            - c2(t3) c2(t2-t1), with m4 and c2 the sample moments of x~
 *            formed the same way (the zero-mean moment-to-cumulant relation;
 *            Section 1 defines cumulants through the moments).
 * Layouts.   c3: (2M+1)^2 row-major float64, lag (w1,w2) at
 *            (w1+M)*(2M+1) + (w2+M).  By default only the hexagon
 *            |w1-w2| <= M is filled and the two corners of the square are
 *            0; with HOS_FULL_SQUARE every lag |w1|,|w2| <= M holds its
 *            sample cumulant.
 *            B: nfft x nfft interleaved complex128, row-major, frequency
 *            (k1,k2) at k1*nfft + k2, unshifted.
 *            B(k1,k2) = sum_w W(w) c3(w) exp(-2 pi i (k1 w1 + k2 w2)/nfft),
 *            unnormalised, with the sign of the DFT in Algorithm DBS's part DFT,
 *            the sum over every lag |w1|,|w2| <= M (the sample cumulant at
 *            the corners is computed whenever W is nonzero there: always
 *            for HOS_WIN_NONE and HOS_WIN_PARZEN_SEPARABLE, never needed for
 *            HOS_WIN_PARZEN, which vanishes at |w1-w2| >= M).
 *            With HOS_PD_ONLY: only the principal domain 0 <= k2 <= k1,
 *            k1+k2 < nfft/2, row-major in (k1, then k2), packed.
 *            c4: (2M+1)^3 row-major float64, lag (t1,t2,t3) at
 *            ((t1+M)*(2M+1) + (t2+M))*(2M+1) + (t3+M); lags whose span
 *            max(0,t1,t2,t3) - min(0,t1,t2,t3) exceeds M are 0.
 *            T: nfft^3 interleaved complex128, frequency (k1,k2,k3) at
 *            (k1*nfft + k2)*nfft + k3, unshifted, the 3-D analogue of B.
 * Threading. Calls are re-entrant; concurrent calls must use distinct
 *            workspaces.
 */
#ifndef HOS_H
#define HOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque HIP stream handle (the same type as in the HIP runtime headers). */
typedef struct ihipStream_t *hipStream_t;

#define HOS_VERSION 10000 /* 1.0.0 */

/* Status codes. */
typedef enum hos_status {
    HOS_OK = 0,
    HOS_EINVAL = -1,       /* an argument is out of range, null or misaligned */
    HOS_EWORKSPACE = -2,   /* ws_bytes is smaller than the workspace query   */
    HOS_EDEVICE = -3,      /* a HIP call or kernel launch failed              */
    HOS_ENODEVICE = -4,    /* no usable gfx950 device is visible              */
    HOS_EUNSUPPORTED = -5, /* valid request the library does not implement   */
    HOS_ESCRATCH = -6      /* the request needs more than the fixed scratch of
                              hos_bispectrum_noalloc (HOS_NOALLOC_SCRATCH_BYTES) */
} hos_status;

/* Element type of the input series. */
typedef enum hos_dtype { HOS_F32 = 0, HOS_F64 = 1 } hos_dtype;

/* Lag window applied before the DFT.  The paper smooths in frequency with
 * an M3 x M3 box (Algorithm DBS's box smoothing); this library smooths in the lag
 * domain instead.  HOS_WIN_PARZEN uses the Parzen window d(m) with scale
 * L = M: W3(w1,w2) = d(w1) d(w2) d(w1-w2) for the bispectrum and the
 * product of d over the six pairwise differences of {0,t1,t2,t3} for the
 * trispectrum.  HOS_WIN_PARZEN_SEPARABLE is the product over the lags only
 * (the alternative reading): d(w1) d(w2), resp. d(t1) d(t2) d(t3). */
typedef enum hos_window {
    HOS_WIN_NONE = 0,
    HOS_WIN_PARZEN = 1,
    HOS_WIN_PARZEN_SEPARABLE = 2   /* d(w1) d(w2); trispectrum d(t1) d(t2) d(t3) */
} hos_window;

/* Arithmetic of the cumulant contraction.  Moments, scaling, cross-tile
 * reductions, windows and DFTs are FP64 on every path.
 *   HOS_PATH_FP32        FP32 matrix-core products and FP32 accumulation;
 *   HOS_PATH_SPLIT_FP16  each operand split into FP16 hi + lo, three
 *                        FP16 products (hi*hi + hi*lo + lo*hi), FP32
 *                        accumulation;
 *   HOS_PATH_SPLIT_BF16  the same with BF16 halves.
 * FP32 partial sums are flushed into FP64 every 512 samples (every 1024 in
 * the third-order contraction's split paths for M >= 96). */
typedef enum hos_path {
    HOS_PATH_FP32 = 0,
    HOS_PATH_SPLIT_FP16 = 1,
    HOS_PATH_SPLIT_BF16 = 2
} hos_path;

/* Flags. */
#define HOS_NO_CENTER 1u     /* use x as given (no mean removal); for tests      */
#define HOS_FULL_SQUARE 2u   /* hos_bispectrum[_streamed]: fill c3's corners     */
#define HOS_PD_ONLY 4u       /* hos_bispectrum: B on the principal domain only   */
#define HOS_PLAN_ADJOINT 16u /* batch plan flag: also lay out the adjoint buffers */
#define HOS_PLAN_SEGMENTS 32u /* batch plan flag: lay out hos_bispectrum_segments' buffers */

/* Human-readable text for a status code (static storage). */
const char *hos_strerror(int status);

/* HOS_VERSION of the loaded library. */
int hos_version(void);

/* HOS_OK if a gfx950 device is current, else HOS_ENODEVICE / HOS_EDEVICE. */
int hos_device_check(void);

/*
 * Workspace size for hos_bispectrum.  It does not depend on the window:
 * the corner lags some windows need reuse the partial-sum region.
 *   n      series length, n >= 2.
 *   M      maximum lag, 0 <= M < n.
 *   nfft   DFT size per axis, or 0 when no spectrum is requested.
 *   path   hos_path.
 *   flags  HOS_* flags.
 *   bytes  (host) receives the size in bytes.
 * Returns HOS_EINVAL on a bad argument (same rules as hos_bispectrum).
 */
int hos_bispectrum_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path,
                             uint32_t flags, size_t *bytes);

/*
 * Third-order cumulant and smoothed bispectrum of one series
 * (Section 1 "Problem Statement"; indirect method).
 *   x        device, n elements of dtype (HOS_F32 / HOS_F64), 4/8-byte aligned.
 *   M        maximum lag, 0 <= M < n.
 *   window   hos_window.
 *   nfft     DFT size per axis, 2 <= nfft <= 4096, nfft = 2^a 3^b 5^c;
 *            nfft >= 2M with either Parzen window (it vanishes at |w| = M),
 *            nfft >= 2M+1 with HOS_WIN_NONE; ignored when B is NULL.
 *   path     hos_path.
 *   flags    HOS_NO_CENTER, HOS_FULL_SQUARE (c3 at the corners |w1-w2| > M
 *            too: the sums over F' = {0 <= b <= M, M < a <= b + M} of the
 *            sorted offsets {0, b, a}, computed by a second contraction of
 *            the same shape), HOS_PD_ONLY (B on the principal domain).
 *   c3       device, (2M+1)^2 float64 (layout above), or NULL.
 *   B        device, nfft^2 complex128 (layout above), or with HOS_PD_ONLY
 *            npd complex128, npd = sum over k1 = 0 .. H of
 *            max(0, min(k1, H - k1) + 1), H = floor((nfft-1)/2); or NULL.
 *   ws       device workspace of at least hos_bispectrum_workspace() bytes
 *            (queried with the same flags), 256-byte aligned; its contents
 *            on entry do not matter.
 * At least one of c3 and B must be non-NULL.
 */
int hos_bispectrum(const void *x, int32_t dtype, int64_t n, int32_t M,
                   int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                   double *c3, double *B, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/*
 * hos_bispectrum with per-stage timing, for profiling.  Same arguments and
 * results; additionally records HIP events around each stage on `stream`,
 * WAITS for the stream, and writes the elapsed milliseconds to stage_ms
 * (host, 8 floats): [0] mean/range pass, [1] operand preparation,
 * [2] contraction, [3] leftover diagonal sums, [4] partial reduction (with
 * the corner contraction and its reduction when the square is computed),
 * [5] mirror, window and the DFT along k2 (+ twiddles), [6] the DFT along
 * k1, [7] total.  Creates and
 * destroys its own events (no device memory is allocated).
 */
int hos_bispectrum_timed(const void *x, int32_t dtype, int64_t n, int32_t M,
                         int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                         double *c3, double *B, void *ws, size_t ws_bytes,
                         hipStream_t stream, float *stage_ms);

/*
 * hos_bispectrum without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.
 *
 * Arguments and results as for hos_bispectrum.  The workspace is a device
 * array of HOS_NOALLOC_SCRATCH_BYTES inside the library, one per device,
 * held from the library's first use on that device until the process ends.
 * The call makes no hipMalloc/hipFree and no allocating library call; its
 * first call on a device looks up that device's array (hipGetSymbolAddress).
 * Requests whose hos_bispectrum_workspace size exceeds
 * HOS_NOALLOC_SCRATCH_BYTES return HOS_ESCRATCH before any HIP call (at
 * n = 2^20, M = 512: 86 MiB on the FP32 path, 118 MiB on the split paths).
 * Every call on one device shares that device's array: calls that overlap
 * in time on one device race and must be serialised by the caller (one
 * stream, or synchronisation between them).  Nothing in the array needs to
 * be zero on entry; it keeps the last call's contents.
 */
#define HOS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20) /* 128 MiB per device */
int hos_bispectrum_noalloc(const void *x, int32_t dtype, int64_t n, int32_t M,
                           int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                           double *c3, double *B, hipStream_t stream);

/*
 * Host-only introspection of the contraction plan (no HIP call, no device
 * needed).  info (host) receives, in order: persistent workgroups G,
 * partial slots per workgroup, tile rows, chunks per tile, 32-blocks per
 * tile side, 32-block rows, leftover diagonal sums, padded length, total
 * schedule cost, workspace bytes.  ninfo >= 10.  HOS_EINVAL on bad sizes.
 */
int hos_c3_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo);

/*
 * Host-only replay of the contraction's work split, for testing without a
 * GPU.  For every (tile, chunk) pair k in schedule order (cap >= tiles x
 * chunks, all arrays host): owner[k] = workgroup that processes it (-1 none,
 * -2 more than one), slot[k] = partial slot it writes (-3 out of range),
 * rslot[k] = slot the reduction reads for it (-4 inconsistent owner).
 */
int hos_c3_schedule(int64_t n, int32_t M, int32_t path, int64_t *owner, int64_t *slot,
                    int64_t *rslot, int64_t cap);

/*
 * Workspace size for hos_trispectrum; arguments as for
 * hos_bispectrum_workspace, with the limits of hos_trispectrum.  T folds
 * the c4 cube: with c4 = NULL the workspace holds that cube ((2M+1)^3
 * float64; the size for nfft > 0 includes it).
 */
int hos_trispectrum_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path,
                              uint32_t flags, size_t *bytes);

/*
 * Fourth-order cumulant and smoothed trispectrum of one series (Section 1
 * "Problem Statement"; the indirect method one order up, as Section 3's
 * k-th order generalisation describes).  Arguments as for hos_bispectrum,
 * except:
 *   M        maximum lag, 0 <= M <= 127 and M < n.
 *   nfft     DFT size per axis, 2 <= nfft <= 512, nfft = 2^a 3^b 5^c,
 *            nfft >= 2M (Parzen) / 2M+1 (no window); ignored when T is NULL.
 *   c4       device, (2M+1)^3 float64 (layout above), or NULL.
 *   T        device, nfft^3 complex128 (layout above), or NULL.
 * At least one of c4 and T must be non-NULL.  The lag window must be
 * HOS_WIN_PARZEN: the product of d(m), scale L = M, over the six pairwise
 * differences of {0, t1, t2, t3}, which vanishes wherever the span exceeds
 * M.  The other windows are nonzero at lags of span up to 2M, which this
 * contraction does not cover: they return HOS_EUNSUPPORTED.
 */
int hos_trispectrum(const void *x, int32_t dtype, int64_t n, int32_t M,
                    int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                    double *c4, double *T, void *ws, size_t ws_bytes,
                    hipStream_t stream);

/*
 * hos_trispectrum with per-stage timing (see hos_bispectrum_timed): WAITS
 * for the stream and writes 7 floats of milliseconds to stage_ms (host):
 * [0] mean/range pass, [1] operand preparation, [2] contraction,
 * [3] partial reduction + second-order moments, [4] cumulant assembly,
 * window, fold and the DFT along k3 (+ twiddles), [5] the DFTs along k2 and
 * k1, [6] total.
 */
int hos_trispectrum_timed(const void *x, int32_t dtype, int64_t n, int32_t M,
                          int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                          double *c4, double *T, void *ws, size_t ws_bytes,
                          hipStream_t stream, float *stage_ms);

/*
 * Host-only plan of the fourth-order contraction (no HIP call).  info
 * (host) receives: lag pairs, 32-pair blocks, 32-column blocks, staged
 * window samples, sample-axis ranges, chunks per range, chunks, workspace
 * bytes.  ninfo >= 8.  HOS_EINVAL on bad sizes.
 */
int hos_c4_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo);

/*
 * A record in host memory, streamed (the memory frugality of Section 3's
 * window-sum theorems, for the indirect estimator): the same c3 and B as
 * hos_bispectrum on the whole record, computed through a device workspace
 * whose size depends on the piece length P and M but not on n.  The record
 * is read twice: first for its FP64 mean and scale, then in pieces of P
 * samples, each with the M samples after it (2M when the square's corners
 * are computed: HOS_FULL_SQUARE, or a window that is nonzero there), whose
 * sums are added to a running FP64 table.  The first pass reads a record
 * in pinned host memory that the device maps at the same address
 * (hipHostMalloc, or hipHostRegister with mapping) in place, in one launch;
 * any other record it copies piece by piece.  The copies run on a copy
 * stream of the library's own (one per device, made at the first call and
 * kept until the process ends) into two staging buffers of the workspace,
 * so a piece's copy overlaps the kernels of the one before; events order
 * them against `stream`, whose completion implies every copy's.
 *   x_host  host memory, n samples, HOS_F32 or HOS_F64.  With pinned memory
 *           the call returns once everything is queued; the record must
 *           stay valid and unchanged until `stream` has passed the call.
 *           Pageable memory works too (the runtime stages it, and the call
 *           returns about when the last piece's copy has been taken).
 *   piece   P: a multiple of 1024, >= 4096, >= M.
 *   c3, B, window, nfft, path: as hos_bispectrum (device outputs).
 *   flags   HOS_NO_CENTER, HOS_FULL_SQUARE (as hos_bispectrum).
 * Workspace: hos_bispectrum_streamed_workspace (dtype sets the size of the
 * piece buffer; the size covers the corners whatever the window).  Results equal hos_bispectrum's up to the order of FP64
 * additions.
 */
int hos_bispectrum_streamed_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path,
                                      int32_t dtype, int64_t piece, size_t *bytes);
int hos_bispectrum_streamed(const void *x_host, int32_t dtype, int64_t n, int32_t M,
                            int32_t window, int32_t nfft, int32_t path, uint32_t flags,
                            int64_t piece, double *c3, double *B, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/*
 * ------------------------------------------------------------------------
 * Order five (the k-th order generalisation of Section 3 at k = 5).
 *
 * m5(t1..t4) = (1/n) sum_t x~_t x~_{t+t1} x~_{t+t2} x~_{t+t3} x~_{t+t4} (same
 * index range and normalisation as c3), and for the zero-mean series the
 * moment-to-cumulant relation keeps besides m5 only the splits of the five
 * offsets {0, t1, t2, t3, t4} into a pair and a triple:
 *   c5 = m5 - sum over the ten pairs {j,k} of c2(o_k - o_j) c3(the other three),
 * with c2 and c3 the sample cumulants of the same series.  Lags whose span
 * max - min of {0, t1..t4} exceeds M are 0.  Window: HOS_WIN_PARZEN, d over
 * the ten pairwise differences of the offsets (L = M), which vanishes
 * wherever the span exceeds M; the other windows would need lags of span up
 * to 2M and return HOS_EUNSUPPORTED.
 *   Q(k1..k4) = sum_t W5(t) c5(t) exp(-2 pi i <k, t> / N).
 * Outputs: c5 (2M+1)^4 float64 row-major, lag t at t+M per axis; Q N^4
 * interleaved complex128, unshifted.  Either may be NULL (not both).  Limits:
 * M <= 40, N <= 96 (2, 3, 5-smooth, >= 2M with a window, >= 2M+1 without).
 * The fifth moments come from the matrix cores (rows x_i x_{i+a} x_{i+b}
 * x_{i+c}, 0 <= c <= b <= a <= M, against the columns x_{i+d}, d <= c);
 * c2 and c3 are FP64 sums over the input.  Q folds the c5 cube: with c5 =
 * NULL the workspace holds that cube ((2M+1)^4 float64; the workspace size
 * for nfft > 0 includes it).
 * ------------------------------------------------------------------------
 */
int hos_cumulant5_workspace(int64_t n, int32_t M, int32_t nfft, int32_t path, uint32_t flags,
                            size_t *bytes);
int hos_cumulant5(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                  int32_t nfft, int32_t path, uint32_t flags, double *c5, double *Q, void *ws,
                  size_t ws_bytes, hipStream_t stream);
/* stage_ms (host, 5 floats): moments and operands, contraction, reduction
 * with c2 / c3, the fold and the DFT along the last axis, the DFTs along
 * the other three axes, total.  Synchronises the stream. */
int hos_cumulant5_timed(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                        int32_t nfft, int32_t path, uint32_t flags, double *c5, double *Q,
                        void *ws, size_t ws_bytes, hipStream_t stream, float *stage_ms);
/* Host-only plan of the order-five contraction; info as hos_c4_plan_info
 * (the first entry counts lag triples). */
int hos_c5_plan_info(int64_t n, int32_t M, int32_t path, int64_t *info, int32_t ninfo);

/*
 * ------------------------------------------------------------------------
 * Batches of series.
 *
 * A batch is described by a PLAN built on the host (no device needed):
 * series s has n[s] samples, stored at x + sum_{t<s} n[t] of one packed
 * device array, and maximum lag M[s].  Its DFT size is the smallest
 * 2^a 3^b 5^c >= 2M[s].  The plan lays out
 * the workspace and cuts every series' c3 contraction into work items
 * (series, tile, chunk range) that it assigns to persistent workgroups by
 * the longest-processing-time rule.  The caller copies the plan bytes
 * unchanged to device memory (256-byte aligned) and passes BOTH copies to
 * the batched calls: the host copy sets up the launches, the kernels read
 * the device copy.  A plan may be reused for any number of calls.
 *
 * Outputs are packed in series order: c3 of series s (its (2M+1)^2 block,
 * layout as above) starts at element sum_{t<s} (2M[t]+1)^2; B on the
 * principal domain 0 <= k2 <= k1, k1+k2 < N/2 (Algorithm DBS's raw bispectrum, here on
 * the N grid), in row-major (k1, then k2) order, starts at complex element
 * sum_{t<s} npd(N[t]).  hos_batch_series reports every offset.
 * ------------------------------------------------------------------------
 */

/* Plan and workspace sizes for a batch.  n, M: host arrays of `batch`
 * entries (1 <= batch <= 65535: the series index is a grid dimension of
 * the per-series kernels; n >= 2, 0 <= M < n, DFT size N <= 2048, i.e. M <= 1024 with
 * the Parzen window; M <= 320 with HOS_PLAN_ADJOINT).
 * window: HOS_WIN_PARZEN (batches compute the hexagon only, so the windows
 * that are nonzero at its corners return HOS_EUNSUPPORTED).
 * flags: HOS_NO_CENTER, HOS_PLAN_SEGMENTS (see
 * hos_bispectrum_segments; needs one M for every series), HOS_PLAN_ADJOINT (lay out the
 * buffers hos_bispectrum_loss_bwd needs).  tile_nb: NULL, or a host array
 * of `batch` tile choices for the contraction, 0 = built-in rule, 2 = tiles
 * of 2 x 2 matrix-core blocks (split paths only), 4 = 4 x 4 blocks; this is
 * what the package's tuner (paper_1805_11775_amd.tune) chooses per lag.
 * Host only. */
int hos_batch_plan_size(int32_t batch, const int64_t *n, const int32_t *M, int32_t window,
                        int32_t path, uint32_t flags, const int32_t *tile_nb,
                        size_t *plan_bytes, size_t *ws_bytes);

/* Writes the plan into host memory `plan` (8-byte aligned, plan_bytes from
 * hos_batch_plan_size with the same arguments).  Host only. */
int hos_batch_plan(int32_t batch, const int64_t *n, const int32_t *M, int32_t window,
                   int32_t path, uint32_t flags, const int32_t *tile_nb, void *plan,
                   size_t plan_bytes);

/* Host-only queries of a plan (host copy).  hos_batch_plan_info: info[0..11]
 * = batch, c3 elements, principal-domain points, input samples, workspace
 * bytes, plan bytes, work items and workgroups of the 2x2- and 4x4-block
 * tile classes (items0, items1, G0, G1), the common M (or -1), the largest
 * principal domain.  hos_batch_series: 8 int64 per series = n, M, N, npd,
 * x offset, c3 offset, B offset, tile class.  hos_batch_items: 8 int64 per
 * work item of class cls (0: 2 x 2 blocks, 1: 4 x 4 blocks, -1: every item)
 * in launch order = class, workgroup, series, tile row, tile column, first
 * chunk, end chunk, partial slot.  The contraction is ONE persistent launch
 * over the items of both classes (G0 = G1 workgroups); a workgroup runs its
 * 4 x 4 items, then its 2 x 2 items. */
int hos_batch_plan_info(const void *plan, int64_t *info, int32_t ninfo);

/*
 * The batch tile tuner (the choice passed to hos_batch_plan as tile_nb),
 * timed on the device.  For every maximum lag Ms[i] and length bucket j
 * (lengths n_edges[j] <= n < n_edges[j+1]) it builds a synthetic batch of
 * `series` uniform(-1, 1) float32 series with lengths spread evenly over the
 * bucket, plans it with every candidate tile (2 and 4 blocks on the split
 * paths, 4 on the FP32 path), builds the operand tables once, and times
 * the contraction launch alone `reps` times (HIP events; the median
 * counts).
 *   path      hos_path.
 *   Ms        host, nM lags, 0 <= M <= 1024, M + 2 < n_edges[nb]; 1 <= nM <= 64.
 *   n_edges   host, nb + 1 increasing lengths (2 <= n <= 2^24); 1 <= nb <= 16.
 *   series    series per synthetic batch, 1 .. 4096; reps 1 .. 100.
 *   ws        device workspace of hos_tune_workspace() bytes, 256-byte aligned.
 *   tile_out  host, nM x nb: the faster tile (2 or 4) per (M, bucket).
 *   ms_out    host, nM x nb x 2: median contraction milliseconds of the
 *             2-block and 4-block tiles (-1 where not a candidate).
 * WAITS for `stream`.  HOS_EINVAL for bad sizes (checked on the host first).
 */
int hos_tune_workspace(int32_t path, const int32_t *Ms, int32_t nM, const int64_t *n_edges,
                       int32_t nb, int32_t series, size_t *bytes);
int hos_tune(int32_t path, const int32_t *Ms, int32_t nM, const int64_t *n_edges, int32_t nb,
             int32_t series, int32_t reps, void *ws, size_t ws_bytes, int32_t *tile_out,
             float *ms_out, hipStream_t stream);
/*
 * Measurement helper (not a step of the estimator): the matrix cores'
 * attainable rate on the current device.  One four-wave workgroup per
 * compute unit issues `iters` rounds of four independent 32 x 32 MFMA ops
 * per wave (v_mfma_f32_32x32x16_f16 / _bf16 for the split paths,
 * v_mfma_f32_32x32x2_f32 for HOS_PATH_FP32) and nothing else; a short
 * warm-up launch precedes the timed one.
 *   iters      1 .. 2^24 (2^19 runs for about 40 ms on MI355X).
 *   ms_out     host: the timed launch's milliseconds (HIP events).
 *   flops_out  host: the FLOP that launch issued (2 x 32 x 32 x k per op).
 * WAITS for `stream`.  Writes no device memory.  HOS_EINVAL for a bad path
 * or count (checked before any HIP call).
 */
int hos_mfma_rate(int32_t path, int32_t iters, float *ms_out, double *flops_out,
                  hipStream_t stream);
int hos_batch_series(const void *plan, int64_t *out, int64_t cap);
int hos_batch_items(const void *plan, int32_t cls, int64_t *out, int64_t cap);

/*
 * Bispectra of every series of a batch in one pass (the estimator of
 * hos_bispectrum applied to each series; window and path from the plan).
 *   x          device, packed series of dtype.
 *   plan_host  the host plan; plan_dev its device copy.
 *   c3         device, packed c3 blocks (plan_info[1] float64), or NULL.
 *   B_pd       device, packed principal-domain spectra (plan_info[2]
 *              complex128), or NULL.  At least one must be non-NULL.
 *   ws         device workspace of plan_info[4] bytes, 256-byte aligned.
 */
int hos_bispectrum_batched(const void *x, int32_t dtype, const void *plan_host,
                           const void *plan_dev, double *c3, double *B_pd, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/*
 * hos_bispectrum_batched with per-stage timing (HIP events on `stream`);
 * WAITS for the stream and writes 5 floats of milliseconds to stage_ms
 * (host): [0] mean/range and operand tables, [1] contraction, [2] partial
 * and diagonal sums, [3] c3 output and spectra, [4] total.  Used by the
 * tile tuner to time the contraction on its own.
 */
int hos_bispectrum_batched_timed(const void *x, int32_t dtype, const void *plan_host,
                                 const void *plan_dev, double *c3, double *B_pd, void *ws,
                                 size_t ws_bytes, hipStream_t stream, float *stage_ms);

/*
 * Bispectrum-matching loss over a batch whose series share one M:
 *   L = sum_s sum_{k in PD} |B_s(k) - target(k)|^2.
 *   target_pd  device, npd complex128 (the principal domain of the common N).
 *   B_pd       device, receives the batch's principal-domain spectra.
 *   loss       device, one float64.
 */
int hos_bispectrum_loss_fwd(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, const double *target_pd, double *B_pd,
                            double *loss, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Gradient of the loss: dx = dL * dL/dx for every sample of every series,
 * with B_pd from hos_bispectrum_loss_fwd on the same x and plan, and dL a
 * device float64 (the upstream gradient).  The plan must have been made
 * with HOS_PLAN_ADJOINT.  dx: device, same dtype and packing as x.  The
 * product terms are recomputed from x; nothing of the forward pass but B_pd
 * is needed.
 */
int hos_bispectrum_loss_bwd(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, const double *B_pd, const double *target_pd,
                            const double *dL, void *dx, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/*
 * Segment averaging (Algorithm DBS's split into parts, per-part mean removal and average over parts, around the cumulant):
 * the series of a batch plan are the segments of one record, each centred on
 * its own mean; their third cumulants are averaged,
 *   c3(w) = (1/S) sum_s c3_s(w),
 * and the average is windowed and transformed as by hos_bispectrum.  The
 * plan must have been made with HOS_PLAN_SEGMENTS, every series with the same
 * M (then one DFT size N, the plan's); x is the packed input, so segments of
 * P consecutive samples of one record are a plan with n[s] = P.
 *   c3  device, (2M+1)^2 float64 (as hos_bispectrum), or NULL.
 *   B   device, N x N interleaved complex128 (as hos_bispectrum), or NULL
 *       (not both NULL).
 * Returns HOS_EINVAL for a plan without the flag or without one M.
 */
int hos_bispectrum_segments(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, double *c3, double *B, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/*
 * ------------------------------------------------------------------------
 * The direct method (Algorithm DBS, Section 1) with the window-sum smoothing
 * of Section 3 (Algorithm WS, Theorem directseq).
 *
 * The first K = floor(n / P) * P samples are cut into K parts of P samples
 * (trailing samples are not used).  Each part loses its own mean (FP64;
 * kept with HOS_NO_CENTER) and gets a P-point DFT
 *     F_i(k) = sum_u x_i(u) exp(-2 pi i u k / P).
 * The raw bispectrum of a part is F_i(k1) F_i(k2) conj F_i(k1 + k2) / P
 * (indices modulo P; the conjugate on the third factor is what
 * makes the estimate agree with the Fourier transform of the third
 * moment).  It is averaged over the M3 x M3 box of offsets
 * n1, n2 in [-floor(M3/2), M3 - 1 - floor(M3/2)] around each point, indices
 * modulo P (for even M3 this is the printed range -M3/2 .. M3/2-1), and
 * over the K parts.  Every value is computed in FP64.
 *
 * Output: the principal domain 0 <= k2 <= k1, k1 + k2 < P/2 of the P grid,
 * row-major in (k1, k2) -- row k1 (0 <= k1 <= H = floor((P-1)/2)) holds
 * k2 = 0 .. min(k1, H - k1) -- as interleaved complex128.
 *
 * Limits: 2 <= P <= 65536 with no prime factor but 2, 3, 5; n >= P;
 * 1 <= M3 <= min(P, 2048).  Cost: O(n log P) for the DFTs, O(K) per output
 * for the part sums (K >= 2), and O(1) per output for the smoothing,
 * independent of M3.
 * ------------------------------------------------------------------------
 */

/* Workspace bytes (host-only).  HOS_EINVAL on bad sizes. */
int hos_dbs_workspace(int64_t n, int32_t P, int32_t M3, size_t *bytes);

/*
 * x: device, n samples (HOS_F32 or HOS_F64).  flags: 0 or HOS_NO_CENTER.
 * B_pd: device, 16-byte aligned, npd complex128 (npd from
 * hos_dbs_plan_info).  ws: device, 256-byte aligned, >= hos_dbs_workspace
 * bytes; no contents are assumed on entry.  Asynchronous on `stream`;
 * nothing is allocated.  Deterministic: a fixed summation order throughout.
 * Returns HOS_EINVAL / HOS_EWORKSPACE before any device work, HOS_EDEVICE
 * if a launch fails.
 */
int hos_dbs(const void *x, int32_t dtype, int64_t n, int32_t P, int32_t M3, uint32_t flags,
            double *B_pd, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * hos_dbs with stage timing (synchronises the stream): stage_ms (host, 4
 * floats) receives the part means and DFTs, the part sums (0 when K = 1),
 * the smoothing, and the total, in milliseconds.  Two tuning arguments
 * (0: the built-in rule): seg_rows > 0 sets the output rows per smoothing
 * workgroup; strip_w in {512, 1024, 2048}, >= M3, sets the widened strip
 * width.  Results differ from hos_dbs by rounding only.  The workspace must
 * hold the byte count hos_dbs_plan_info gives for the same arguments.
 */
int hos_dbs_timed(const void *x, int32_t dtype, int64_t n, int32_t P, int32_t M3,
                  uint32_t flags, double *B_pd, void *ws, size_t ws_bytes, hipStream_t stream,
                  int32_t seg_rows, int32_t strip_w, float *stage_ms);

/*
 * Host-only plan (no HIP call), for the tuning arguments of hos_dbs_timed
 * (0, 0: the plan of hos_dbs).  info (host, ninfo >= 16) receives: K,
 * mode (0: products formed from the spectrum, K = 1; 1: part sums first),
 * P1, P2 (the part DFT as P1 x P2 passes; P2 = 1 for one pass), widened
 * strip width, output strip width, strips, rows per smoothing workgroup,
 * smoothing workgroups, part-sum rectangle rows and columns, part groups,
 * parts per group, principal-domain points npd, workspace bytes, and the
 * strips' rows in total.
 */
int hos_dbs_plan_info(int64_t n, int32_t P, int32_t M3, int32_t seg_rows, int32_t strip_w,
                      int64_t *info, int32_t ninfo);

#ifdef __cplusplus
}
#endif

#endif /* HOS_H */
