// hos_internal.h -- internal plan, workspace layout and launch declarations
// of the gfx950 higher-order-spectra library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hos.h"

namespace hos {

// ---------------------------------------------------------------------------
// Contraction geometry.
//
// The third-order sums over the fundamental region F = {0 <= b <= a <= M}
//     C[a][b] = sum_i x_i x_{i+a} x_{i+b}
// are computed as a matrix product over the sample index i: for the row
// r = a - 1 (a = 1..M) the product row Y[r][i] = x_i x_{i+r+1} meets the
// Hankel operand T[i][b] = x_{i+b}.  Rows and columns are cut into 32 x 32
// matrix-core blocks; block (R, B) is needed iff B <= R.  Inside a diagonal
// block the entries with b <= r + 1 are kept, which covers every (a, b) of F
// except the diagonal entries C[a][a] for a = 0 and a = 32k; those few
// sums are computed separately (k_diag_dot).
//
// Blocks are grouped into square workgroup tiles of TS = 32*NB samples per
// side (NB = 2 or 4 blocks); a workgroup has NB waves and wave w owns the
// 32-row strip w of the tile against all NB column blocks.  The sample
// axis is cut into chunks of KC samples; a "chunk" of a tile is the unit of
// work.  Chunks are spread over a fixed number G of persistent workgroups
// by a weighted contiguous split of the flattened (tile, chunk) sequence
// ("stream-K"): each workgroup owns the chunks whose start cost falls in its
// cost range and writes one FP64 partial tile per tile it touches, so the
// cross-workgroup reduction is a fixed-order sum (deterministic).
// ---------------------------------------------------------------------------
constexpr int KC = 512;           // samples per (sub-)chunk; FP32 -> FP64 flush period
constexpr int GROUP = 16;         // samples per matrix-core k-group
constexpr int WG_THREADS = 256;   // 4 waves of 64

struct SkGeom {
    int32_t TR;     // tile rows (and columns) of the triangle
    int32_t cf;     // cost of one chunk of an off-diagonal tile
    int32_t cd;     // cost of one chunk of a diagonal tile
    int32_t G;      // persistent workgroups
    int64_t C;      // chunks per tile
    int64_t ctot;   // total cost
};

struct SkPos {
    int32_t R;      // tile row
    int32_t Cc;     // tile column (Cc <= R)
    int64_t c;      // chunk index within the tile
};

__host__ __device__ inline int64_t sk_row_prefix(const SkGeom &g, int64_t R)
{
    // cost per chunk-column of all tiles in rows < R (R-1 full + 1 diagonal each)
    return (R * (R - 1) / 2) * g.cf + R * g.cd;
}

__host__ __device__ inline int sk_tile_cost(const SkGeom &g, int R, int Cc)
{
    return Cc == R ? g.cd : g.cf;
}

__host__ __device__ inline int64_t sk_tile_index(int R, int Cc)
{
    return (int64_t)R * (R + 1) / 2 + Cc;
}

__host__ __device__ inline int64_t sk_chunk_start(const SkGeom &g, int R, int Cc,
                                                  int64_t c)
{
    int64_t tile_prefix = sk_row_prefix(g, R) + (int64_t)Cc * g.cf;
    return tile_prefix * g.C + c * sk_tile_cost(g, R, Cc);
}

__host__ __device__ inline int64_t sk_wg_start(const SkGeom &g, int64_t w)
{
    return w * g.ctot / g.G;
}

// Workgroup owning the chunk that starts at cost S.
__host__ __device__ inline int64_t sk_owner(const SkGeom &g, int64_t S)
{
    return ((S + 1) * g.G - 1) / g.ctot;
}

// Step to the next chunk in (row, column, chunk) order; false past the end.
__host__ __device__ inline bool sk_next(const SkGeom &g, SkPos &p)
{
    if (++p.c < g.C)
        return true;
    p.c = 0;
    if (p.Cc < p.R) {
        ++p.Cc;
        return true;
    }
    ++p.R;
    p.Cc = 0;
    return p.R < g.TR;
}

// First chunk whose start cost is >= S; false if there is none.
__host__ __device__ inline bool sk_first_chunk(const SkGeom &g, int64_t S, SkPos &p)
{
    if (S >= sk_row_prefix(g, g.TR) * g.C)
        return false;
    int R = 0;
    while (R + 1 < g.TR && sk_row_prefix(g, R + 1) * g.C <= S)
        ++R;
    int64_t u = S - sk_row_prefix(g, R) * g.C;
    int64_t full_span = (int64_t)R * g.cf * g.C;
    int Cc;
    int64_t off;
    int cost;
    if (u < full_span) {
        Cc = (int)(u / ((int64_t)g.cf * g.C));
        off = u - (int64_t)Cc * g.cf * g.C;
        cost = g.cf;
    } else {
        Cc = R;
        off = u - full_span;
        cost = g.cd;
    }
    p.R = R;
    p.Cc = Cc;
    p.c = (off + cost - 1) / cost;
    if (p.c >= g.C) {
        p.c = g.C - 1;
        return sk_next(g, p);
    }
    return true;
}

// Upper bound on the number of tiles one workgroup's cost range can touch.
inline int64_t sk_max_segments(const SkGeom &g)
{
    int64_t span = (g.ctot + g.G - 1) / g.G;
    int64_t min_tile = (int64_t)(g.cd < g.cf ? g.cd : g.cf) * g.C;
    return (span > 0 ? (span - 1) / min_tile : 0) + 2;
}

// ---------------------------------------------------------------------------
// Series preparation shared by both estimators: the mean/range pass and the
// operand tables (all workspace offsets 256-byte aligned).
// ---------------------------------------------------------------------------
struct SeriesPlan {
    int64_t n;
    int32_t M;
    int32_t path;      // hos_path
    int32_t scale_top; // max|x~| * s lies in [2^(top-1), 2^top)
    int64_t npad;      // padded series length (multiple of 64)
    size_t off_stats, off_mpart, off_xf, off_win4, off_win8h, off_win8l;
};

// Bispectrum plan and workspace layout.
struct C3Plan : SeriesPlan {
    int32_t NB;        // 32-blocks per tile side (2 or 4) = waves per workgroup
    int32_t TS;        // tile side in samples (32 * NB)
    int32_t NBR;       // 32-block rows: rows r = 0 .. M-1
    int32_t amax;      // largest span in the table: M (hexagon) or 2M (square)
    int32_t nleft;     // leftover diagonal sums C[a][a], a = 0 and a = 32k <= M
    int32_t dot_blocks;// workgroups per leftover sum
    int64_t smax;      // partial slots per workgroup
    SkGeom sk;
    size_t off_part, off_tfirst, off_cfull, off_dpart, off_twid, off_bfull, total;
};

// Trispectrum plan.  The lag pairs (a, b), 0 <= b <= a <= M, are numbered
// with b ascending, then a; P = (M+1)(M+2)/2 pairs in RB blocks of 32.
// The sample axis is split into S ranges of CPS chunks; workgroup (x, s)
// runs pair blocks 4x .. 4x+3 over range s.
struct C4Plan : SeriesPlan {
    int32_t ord;       // 4 (trispectrum) or 5 (order five: P rows are lag triples)
    int32_t P;         // lag pairs
    int32_t RB;        // 32-pair blocks
    int32_t NCB;       // 32-column blocks of the third lag c = 0..M
    int32_t WX;        // staged window beyond the chunk, in samples
    int32_t S;         // sample-axis ranges
    int32_t CPS;       // chunks per range
    int32_t dot_blocks;// workgroups per c2 lag
    int32_t c3_blocks; // order five: workgroups of the c3 sums (k_c3_dot)
    int64_t C;         // chunks of KC samples
    size_t off_part, off_m4, off_c2part, off_c2, off_twid, total;
    size_t off_c3part, off_c3tab;   // order five: third-order corrections
    size_t off_cube;                // with a spectrum: the (2M+1)^3 c4 / (2M+1)^4 c5 cube
};

constexpr int C4_MAX_M = 127;      // 4 column blocks per pair block
constexpr int C5_MAX_M = 40;       // order five: (2M+1)^4 lags of output
constexpr int C5_MAX_NFFT = 96;    // order five: N^4 complex128 spectrum
constexpr int C3D_BS = 512;        // order five: samples per step of k_c3_dot
constexpr int C3D_MAX_WG = 1024;   // its workgroups (each strides over sample blocks)
constexpr int C4_MAX_NFFT = 512;   // N^3 complex128 <= 2 GiB

constexpr int MOM_BLOCKS = 256;     // blocks of the moments pass
constexpr int SK_MAX_WG = 256;      // persistent workgroups of the contraction

// corners: also the square's corner lags (spans a = M+1 .. 2M, kept in the
// table's upper triangle; their contraction reuses the partial-sum region);
// full_grid: stage the N x N spectrum in the workspace (for a
// principal-domain-only output).
int make_c3_plan(int64_t n, int32_t M, int32_t path, int32_t nfft, C3Plan &p,
                 bool corners = false, bool full_grid = false);
// Host-side validation of a hos_bispectrum call (all but the workspace) and
// its plan; no HIP call.
int bispectrum_check(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                     int32_t nfft, int32_t path, uint32_t flags, const double *c3,
                     const double *B, C3Plan &p);
// Validation, plan and launch sequence of hos_bispectrum on the workspace
// `ws` (`ev`: 8 stage events or NULL).
int bispectrum_run(const void *x, int32_t dtype, int64_t n, int32_t M, int32_t window,
                   int32_t nfft, int32_t path, uint32_t flags, double *c3, double *B,
                   void *ws, size_t ws_bytes, hipStream_t stream, hipEvent_t *ev);
int make_c4_plan(int64_t n, int32_t M, int32_t path, int32_t nfft, C4Plan &p, int ord);
int c4_window_entries(int M);

// ---------------------------------------------------------------------------
// Batches.  A host-built plan ("blob", copied unchanged to device memory by
// the caller) describes every series and the contraction's work items.
// Series s occupies samples [x_off, x_off + n) of the packed input and a
// region of the workspace at ws_off; all offsets inside it are bytes.
// ---------------------------------------------------------------------------
struct SeriesDesc {
    int64_t n, x_off, ws_off;
    int64_t c3_off;       // first element of its (2M+1)^2 block of the packed c3
    int64_t pd_off;       // first complex element of its principal-domain block
    int64_t grid_off;     // byte offset (from the workspace base) of its N x N grid
    int64_t npad;         // table entries from sample 0 (zero beyond n)
    int64_t lpad;         // zero table entries before sample 0
    int32_t M, N, NB, NBR, TR, nleft, npd, group, KP, cls;
    int64_t C;            // chunks of c3_stage_len(path, NB) samples
    // byte offsets inside the series region; table offsets point at sample 0
    int64_t o_stats, o_mpart, o_xf, o_win4, o_win8h, o_win8l, o_cfull, o_dpart;
    int64_t o_gtil, o_gtab, o_k64, o_kh, o_kl;   // adjoint buffers (plans made for the adjoint)
    int64_t o_msum;       // adjoint: block sums of the gradient for its mean
};

constexpr int ADJ_MEAN_BLOCK = 4096;   // samples per block sum of the gradient's mean

struct C3Item {           // one (series, tile, chunk range) of the contraction
    int32_t series, R, Cc;
    int32_t pad;          // tile class: 1 = 4 x 4 blocks, 0 = 2 x 2 blocks
    int64_t c0, c1;       // chunks [c0, c1)
    int64_t slot;         // partial tile written
};

struct C3TileRef {        // the slots of one (series, tile), summed in order
    int32_t series, R, Cc, nslot;
    int64_t slot0;
};

struct FftGroup {         // series sharing one DFT size, grids contiguous
    int32_t N, count;
    int64_t grid_off;     // byte offset of the first grid
    int64_t twid_off;     // byte offset of the N twiddles
    int64_t first;        // its series: gseries[first .. first + count)
};

constexpr int64_t BATCH_MAGIC = 0x484f53424154434bLL;   // "HOSBATCK"
constexpr int BATCH_CLASSES = 2;                         // tiles of 2 x 2 / 4 x 4 blocks
constexpr int BATCH_MAX_SERIES = 65535;   // series index = grid y of the per-series kernels
constexpr int BATCH_MAX_WG = 256;                        // persistent workgroups, one per CU

struct BatchHeader {
    int64_t magic, blob_bytes, ws_bytes;
    int64_t batch, path, flags, window;
    int64_t momb, dot_blocks;
    int64_t max_n, max_npad, max_lpad, max_M, max_N, max_nleft, max_npd, max_side2, max_KP;
    int64_t uniform_M, uniform_n;   // shared by every series, else -1
    int64_t c3_total, pd_total, x_total;
    int64_t series_off;             // byte offsets of the arrays inside the blob
    int64_t items_off, n_items_all;  // every work item, both classes, in workgroup order
    int64_t n_items[BATCH_CLASSES];  // items per class
    int64_t wgfirst_off, G[BATCH_CLASSES];   // one launch: G[0] = G[1] workgroups
    int64_t tiles_off[BATCH_CLASSES], n_tiles[BATCH_CLASSES];
    int64_t part_off[BATCH_CLASSES];  // byte offsets of the partial arenas in the workspace
    int64_t groups_off, n_groups;
    int64_t gseries_off;            // int32 series indices ordered by DFT group
    int64_t loss_off;               // byte offset of the per-series loss partials
    int64_t seg_off;                // segments: averaged table, its stats, twiddles (or 0)
};

// Plan flags (in hos.h: HOS_PLAN_ADJOINT).
int batch_plan(int32_t batch, const int64_t *n, const int32_t *M, int32_t window, int32_t path,
               uint32_t flags, const int32_t *tile_nb, void *blob, size_t blob_bytes,
               BatchHeader *hdr_out);
int device_ok_public();
constexpr int ADJ_MAX_M = 320;     // staged adjoint window <= 81 KB of LDS
constexpr int ADJ_NRB = 8;         // adjoint contraction: 32-row blocks per wave
constexpr int ADJ_ROWS = 4 * 32 * ADJ_NRB;   // rows j per workgroup (four waves)

// ---------------------------------------------------------------------------
// Direct method (Algorithm DBS): K parts of P samples, an M3 x M3 box.
// ---------------------------------------------------------------------------
constexpr int DBS_MAX_P = 65536;       // part length (2, 3, 5-smooth)
constexpr int DBS_MAX_M3 = 2048;       // box side (<= one 2048-column strip)
constexpr int DBS_LDS_FFT = 4096;      // longest part DFT done in one LDS pass
constexpr int DBS_CUS = 256;           // compute units the smoothing grid is sized for

struct DbsGeom {          // what the smoothing kernels need
    int32_t P, M3, lo, hi, H;
    int32_t CPT, W, TW;   // columns per thread, extended and output strip widths
    int32_t NS;           // strips; strip s holds the output rows [s TW, H - s TW]
    int32_t R, NSEG;      // rows per workgroup (of the strips' rows laid end to end), workgroups
    int64_t rows;         // sum of the strips' row counts
    int32_t SC;           // row stride of the part-sum rectangle (S mode)
    double norm;          // 1 / (K P M3^2)
};

struct DbsPlan {
    int64_t n, K;
    int32_t mode;         // 0: K = 1, products from the spectrum; 1: from part sums
    int32_t P1, P2;       // two-pass DFT P = P1 * P2 (P2 = 1: one pass)
    int32_t SR;           // rows of the part-sum rectangle
    int32_t G, Kg;        // part groups of the sums, parts per group
    int64_t npd;          // principal-domain points of the P grid
    DbsGeom g;
    size_t off_mean, off_F, off_T, off_tw, off_tw1, off_tw2, off_S, total;
};

int make_dbs_plan(int64_t n, int32_t P, int32_t M3, int32_t seg_rows, int32_t strip_w,
                  DbsPlan &p);
hipError_t launch_dbs(const void *x, int dtype, uint32_t flags, const DbsPlan &p, double *B_pd,
                      char *ws, hipStream_t s, hipEvent_t *ev);

// Element count of one FP64 partial tile.
inline int64_t tile_elems(int NB) { return (int64_t)(32 * NB) * (32 * NB); }
// Samples of one stream-K chunk of the single-series contraction: two KC
// sub-chunks per staged chunk on the split paths with 4-block tiles, one
// elsewhere (the FP32 path stages through registers; 2-block tiles keep two
// workgroups per CU within the LDS).
__host__ __device__ constexpr int c3_stage_len(int path, int NB)
{
    return (path != HOS_PATH_FP32 && NB == 4) ? 2 * KC : KC;
}

// Samples per staged chunk of the batch contraction: both tile classes of
// the split paths stage 1024 samples (one launch, one LDS layout size).
__host__ __device__ constexpr int batch_stage_len(int path)
{
    return path != HOS_PATH_FP32 ? 2 * KC : KC;
}

// ---------------------------------------------------------------------------
// Launchers (enqueue on `s`, return hipError_t of the last launch).
// ---------------------------------------------------------------------------
hipError_t launch_moments(const void *x, int dtype, int64_t n, uint32_t flags,
                          const SeriesPlan &p, char *ws, hipStream_t s);
hipError_t launch_prep(const void *x, int dtype, const SeriesPlan &p, char *ws,
                       hipStream_t s, int64_t key0 = 0, int64_t nfirst = -1);
hipError_t launch_moments_piece(const void *x, int dtype, int64_t len, int first,
                                const SeriesPlan &p, char *ws, double *acc, hipStream_t s);
hipError_t launch_moments_total(const double *acc, int64_t n, uint32_t flags, int top,
                                double *stats, hipStream_t s);
// region 0: the fundamental region F; region 1: the square's corners (the
// Hankel columns M + 1 samples further on, spans a = M+1 .. 2M).
hipError_t launch_c3_contract(const C3Plan &p, char *ws, hipStream_t s, int region = 0);
hipError_t launch_diag_dot(const void *x, int dtype, const C3Plan &p, char *ws,
                           hipStream_t s, int64_t nfirst = -1);
hipError_t launch_c3_reduce(const C3Plan &p, char *ws, hipStream_t s, int region = 0);
// c3 (lags of span <= c3_amax, 0 beyond) and the row transforms of B from a
// table holding spans <= amax (stats[3] divides it).
hipError_t launch_c3_finish(const C3Plan &p, int window, int nfft, double *c3, int c3_amax,
                            double *B, char *ws, hipStream_t s);
hipError_t launch_c3_finish_table(const double *cfull, const double *stats, int M, int amax,
                                  int window, int nfft, const double2 *tw, double *c3,
                                  int c3_amax, double *B, hipStream_t s);
// B_pd[j] = the j-th principal-domain point (row-major k1, then k2) of the
// N x N grid B.
hipError_t launch_pd_gather(const double *B, int N, double *B_pd, hipStream_t s);
bool bispectrum_needs_corners(int32_t window, uint32_t flags, bool want_B);
hipError_t launch_seg_average(const BatchHeader &hdr, const char *dplan, char *ws,
                              hipStream_t s);
bool fft_size_ok(int N);
hipError_t launch_twiddles(double2 *tw, int N, hipStream_t s);
hipError_t launch_full_rows(const double *cfull, const double *stats, int M, int amax, int N,
                            int window, const double2 *tw, double *B, hipStream_t s);
hipError_t launch_fft_cols(double *B, int N, const double2 *tw, hipStream_t s);
hipError_t launch_tri_lines(const double *c4, int M, int N, int window, const double2 *tw,
                            double *T, hipStream_t s);
hipError_t launch_fft3_tail(double *T, int N, const double2 *tw, hipStream_t s);
hipError_t launch_c4_contract(const C4Plan &p, char *ws, hipStream_t s);
// The adjoint's residual DFT of one size group and its lag weights G into
// each series' lag table (k_fft.hip).
hipError_t launch_adj_gweights(const FftGroup &gr, const SeriesDesc *sd, const int32_t *gser,
                               int window, char *ws, hipStream_t s);
hipError_t launch_pd_spectra(const BatchHeader &h, const char *dplan, int window, char *ws,
                             double *B_pd, hipStream_t s);

// Batched launchers: `hdr` is the host copy of the plan, `dplan` its device
// copy, `ws` the workspace base.
hipError_t launch_batch_prep(const void *x, int dtype, const BatchHeader &hdr,
                             const char *dplan, char *ws, hipStream_t s);
hipError_t launch_batch_contract(const BatchHeader &hdr, const char *dplan, char *ws,
                                 hipStream_t s);
hipError_t launch_batch_reduce(const void *x, int dtype, const BatchHeader &hdr,
                               const char *dplan, char *ws, hipStream_t s);
hipError_t launch_batch_spectra(const BatchHeader &hdr, const char *dplan, int window,
                                double *c3, double *B_pd, char *ws, hipStream_t s);
hipError_t launch_batch_loss(const BatchHeader &hdr, const char *dplan, const double *B_pd,
                             const double *target, double *loss, char *ws, hipStream_t s);
hipError_t launch_batch_adjoint(const void *x, int dtype, const BatchHeader &hdr,
                                const char *dplan, int window, const double *B_pd,
                                const double *target, const double *dL, void *dx, char *ws,
                                hipStream_t s);
hipError_t launch_c4_reduce(const void *x, int dtype, const C4Plan &p, char *ws,
                            hipStream_t s);
hipError_t launch_c4_finish(const C4Plan &p, int window, int nfft, double *c4, double *T,
                            char *ws, hipStream_t s);
hipError_t launch_c5_finish(const C4Plan &p, int window, int nfft, double *c5, double *Q,
                            char *ws, hipStream_t s);
hipError_t launch_fft4_tail(double *Q, int N, const double2 *tw, hipStream_t s);

}  // namespace hos
