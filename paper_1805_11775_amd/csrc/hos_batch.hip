// hos_batch.hip -- batches of series: the host planner and the batched C
// entry points (bispectra of many series of uneven length and lag, and the
// bispectrum-matching loss with its adjoint).
//
// The planner runs on the host only.  It lays out one workspace region per
// series, groups the series by DFT size, and cuts every series' c3
// contraction into work items (series, tile, chunk range).  Items are
// assigned to a fixed number of persistent workgroups by the longest-
// processing-time rule: sorted by cost, each goes to the least-loaded
// workgroup.  Every item writes its own FP64 partial tile; a tile's items
// take consecutive slots, summed in chunk order, so results do not depend on
// which workgroup ran what (bitwise deterministic).
#include <string.h>

#include <algorithm>
#include <queue>
#include <vector>

#include "hos_internal.h"

namespace hos {

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }
static int64_t up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

static bool fft_ok(int N)
{
    if (N < 2 || N > 4096)
        return false;
    int m = N;
    for (int r : {2, 3, 5})
        while (m % r == 0)
            m /= r;
    return m == 1;
}

// Smallest 2^a 3^b 5^c >= need (need >= 2).
static int next_fft(int need)
{
    for (int k = need < 2 ? 2 : need;; ++k)
        if (fft_ok(k))
            return k;
}

static int pd_count(int N)
{
    int c = 0;
    for (int a = 0; a < N; ++a)
        for (int b = 0; b <= a; ++b)
            if (2 * (a + b) < N)
                ++c;
    return c;
}

int batch_plan(int32_t batch, const int64_t *n, const int32_t *M, int32_t window, int32_t path,
               uint32_t flags, const int32_t *tile_nb, void *blob, size_t blob_bytes,
               BatchHeader *hdr_out)
{
    if (batch < 1 || batch > BATCH_MAX_SERIES || !n || !M)
        return HOS_EINVAL;
    if (path != HOS_PATH_FP32 && path != HOS_PATH_SPLIT_FP16 && path != HOS_PATH_SPLIT_BF16)
        return HOS_EINVAL;
    if (window != HOS_WIN_NONE && window != HOS_WIN_PARZEN && window != HOS_WIN_PARZEN_SEPARABLE)
        return HOS_EINVAL;
    if (flags & ~(HOS_NO_CENTER | HOS_PLAN_ADJOINT | HOS_PLAN_SEGMENTS))
        return HOS_EINVAL;
    // batches compute each series' hexagon only: the windows that are nonzero
    // at the square's corners would need the corner sums as well
    if (window != HOS_WIN_PARZEN)
        return HOS_EUNSUPPORTED;
    const bool adj = (flags & HOS_PLAN_ADJOINT) != 0;
    const bool split = path != HOS_PATH_FP32;
    BatchHeader h;
    memset(&h, 0, sizeof(h));
    h.magic = BATCH_MAGIC;
    h.batch = batch;
    h.path = path;
    h.flags = flags;
    h.window = window;
    h.uniform_M = M[0];
    h.uniform_n = n[0];
    for (int s = 0; s < batch; ++s) {
        // n <= 2^31: the operand-table grid spans the longest series in one
        // dimension and must stay inside a launch's 32-bit work-item range
        if (n[s] < 2 || n[s] > ((int64_t)1 << 31) || M[s] < 0 || (int64_t)M[s] >= n[s] ||
            M[s] > 2048)
            return HOS_EINVAL;
        if (adj && M[s] > ADJ_MAX_M)
            return HOS_EINVAL;
        if (tile_nb && tile_nb[s] != 0 && tile_nb[s] != 4 && !(tile_nb[s] == 2 && split))
            return HOS_EINVAL;   // the FP32 path has 4 x 4-block tiles only
        if (M[s] != h.uniform_M)
            h.uniform_M = -1;
        if (n[s] != h.uniform_n)
            h.uniform_n = -1;
        h.max_n = std::max<int64_t>(h.max_n, n[s]);
    }
    // moment blocks per series: one per 4096 samples of the longest series,
    // but no more than about 16384 workgroups in all (a large batch fills
    // the chip with a few blocks per series)
    h.momb = std::min<int64_t>(256, std::max<int64_t>(1, (h.max_n + 4095) / 4096));
    h.momb = std::max<int64_t>(1, std::min<int64_t>(h.momb, (16384 + batch - 1) / batch));
    h.dot_blocks = std::min<int64_t>(64, std::max<int64_t>(1, h.max_n / 4096));

    std::vector<SeriesDesc> sd(batch);
    size_t o = 0;
    int64_t xo = 0, c3o = 0, pdo = 0;
    for (int s = 0; s < batch; ++s) {
        SeriesDesc &d = sd[s];
        memset(&d, 0, sizeof(d));
        d.n = n[s];
        d.M = M[s];
        d.x_off = xo;
        xo += n[s];
        d.c3_off = c3o;
        c3o += (int64_t)(2 * d.M + 1) * (2 * d.M + 1);
        d.N = next_fft(window != HOS_WIN_NONE ? 2 * d.M : 2 * d.M + 1);
        if (d.N > 2048)
            return HOS_EINVAL;   // principal-domain DFTs stage 2048-point sequences
        d.npd = pd_count(d.N);
        d.pd_off = pdo;
        pdo += d.npd;
        d.cls = (d.M >= 96 || !split) ? 1 : 0;
        if (tile_nb && tile_nb[s] != 0)
            d.cls = tile_nb[s] == 4 ? 1 : 0;
        d.NB = d.cls ? 4 : 2;
        d.NBR = (d.M + 31) / 32;
        d.TR = d.NBR > 0 ? (d.NBR + d.NB - 1) / d.NB : 0;
        d.nleft = 1 + d.M / 32;
        const int64_t kcx = batch_stage_len(path);   // samples per chunk, both classes
        d.C = (d.n + kcx - 1) / kcx;
        d.KP = adj ? (int32_t)up(2 * d.M + 1, 32) : 0;
        d.lpad = adj ? up(d.M, 64) : 0;
        int64_t npad = up(d.C * kcx + (int64_t)d.TR * 32 * d.NB + 64, 64);
        if (adj)
            npad = std::max<int64_t>(npad, up(up(d.n, ADJ_ROWS) + ADJ_ROWS + d.KP + 128, 64));
        d.npad = npad;
        const int64_t ent = d.lpad + d.npad;
        d.ws_off = (int64_t)o;
        size_t r = 0;
        d.o_stats = r;  r = a256(r + 64 * sizeof(double));
        d.o_mpart = r;  r = a256(r + (size_t)h.momb * 3 * sizeof(double));
        d.o_xf = r + d.lpad * 4;      r = a256(r + (size_t)ent * 4);
        d.o_win4 = r + d.lpad * 16;   r = a256(r + (size_t)ent * 16);
        if (split) {
            d.o_win8h = r + d.lpad * 16;  r = a256(r + (size_t)ent * 16);
            d.o_win8l = r + d.lpad * 16;  r = a256(r + (size_t)ent * 16);
        }
        d.o_cfull = r;  r = a256(r + (size_t)(d.M + 1) * (d.M + 1) * sizeof(double));
        d.o_dpart = r;  r = a256(r + (size_t)d.nleft * h.dot_blocks * sizeof(double));
        if (adj) {
            const size_t kp2 = (size_t)d.KP * d.KP;
            d.o_gtil = r;  r = a256(r + (size_t)d.n * sizeof(double));
            d.o_gtab = r;  r = a256(r + (size_t)(2 * d.M + 1) * (2 * d.M + 1) * sizeof(double));
            d.o_k64 = r;   r = a256(r + kp2 * sizeof(double));
            d.o_msum = r;
            r = a256(r + (size_t)((d.n + ADJ_MEAN_BLOCK - 1) / ADJ_MEAN_BLOCK) * sizeof(double));
            d.o_kh = r;    r = a256(r + kp2 * (split ? 2 : 4));
            if (split) {
                d.o_kl = r;  r = a256(r + kp2 * 2);
            }
        }
        o += r;
        h.max_npad = std::max<int64_t>(h.max_npad, d.npad);
        h.max_lpad = std::max<int64_t>(h.max_lpad, d.lpad);
        h.max_M = std::max<int64_t>(h.max_M, d.M);
        h.max_N = std::max<int64_t>(h.max_N, d.N);
        h.max_nleft = std::max<int64_t>(h.max_nleft, d.nleft);
        h.max_npd = std::max<int64_t>(h.max_npd, d.npd);
        h.max_side2 = std::max<int64_t>(h.max_side2, (int64_t)(2 * d.M + 1) * (2 * d.M + 1));
        h.max_KP = std::max<int64_t>(h.max_KP, d.KP);
    }
    h.c3_total = c3o;
    h.pd_total = pdo;
    h.x_total = xo;

    // DFT groups: grids of one size contiguous, in series order
    std::vector<int> sizes;
    for (auto &d : sd)
        sizes.push_back(d.N);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    std::vector<FftGroup> groups(sizes.size());
    for (size_t g = 0; g < sizes.size(); ++g) {
        groups[g].N = sizes[g];
        groups[g].count = 0;
        groups[g].twid_off = (int64_t)o;
        o = a256(o + (size_t)sizes[g] * 16);
    }
    for (auto &d : sd) {
        const int g = (int)(std::lower_bound(sizes.begin(), sizes.end(), d.N) - sizes.begin());
        d.group = g;
        groups[g].count++;
    }
    for (auto &gr : groups) {
        gr.grid_off = (int64_t)o;
        o = a256(o + (size_t)gr.count * gr.N * gr.N * 16);
    }
    std::vector<int32_t> gseries;
    {
        std::vector<int> fill(groups.size(), 0);
        for (auto &d : sd) {
            FftGroup &gr = groups[d.group];
            d.grid_off = gr.grid_off + (int64_t)fill[d.group]++ * gr.N * gr.N * 16;
        }
        int64_t first = 0;
        for (size_t g = 0; g < groups.size(); ++g) {
            groups[g].first = first;
            for (int s = 0; s < batch; ++s)
                if (sd[s].group == (int)g)
                    gseries.push_back(s);
            first += groups[g].count;
        }
    }
    h.loss_off = (int64_t)o;
    o = a256(o + (size_t)batch * sizeof(double));
    if (flags & HOS_PLAN_SEGMENTS) {
        if (h.uniform_M < 0)
            return HOS_EINVAL;   // one averaged table needs one M
        const size_t ne = (size_t)(h.uniform_M + 1) * (h.uniform_M + 1);
        h.seg_off = (int64_t)o;  // averaged table and 64 stats, then N twiddles
        o = a256(o + a256((ne + 64) * sizeof(double)) + (size_t)sd[0].N * 16);
    }

    // Contraction work items of both tile classes in ONE list for one
    // persistent launch: every (series, tile) is cut into chunk ranges of
    // about `piece` cost units, and the items go to the workgroups by the
    // longest-processing-time rule.  Cost of one chunk: split paths, 14 for
    // a 4 x 4-block tile (its busiest wave: 4 blocks x 1024 samples) and 5
    // for a 2 x 2-block tile (2 blocks x 512 samples: a quarter of the
    // matrix-core work at twice the product-row work per block; the ratio
    // 2.8 is the one the contraction's timings give on MI355X, e.g. 1 tile
    // of 4 x 4 blocks against 3 tiles of 2 x 2 blocks at M = 128); FP32 path
    // (4 x 4 blocks only, 2 x 2 windows per wave), 4 off and 3 on the
    // diagonal.  Partial slots are numbered per class (one partial arena
    // and tile list per class).
    std::vector<C3Item> items;
    std::vector<int64_t> cost;
    std::vector<int32_t> wgfirst;
    std::vector<C3TileRef> tiles[BATCH_CLASSES];
    auto chunk_cost = [&](int cls, bool diag) -> int {
        if (!split)
            return diag ? 3 : 4;
        return cls ? 14 : 5;
    };
    int64_t units = 0;
    for (auto &d : sd)
        for (int R = 0; R < d.TR; ++R)
            for (int Cc = 0; Cc <= R; ++Cc)
                units += chunk_cost(d.cls, Cc == R) * d.C;
    const int64_t gmax = BATCH_MAX_WG;
    const int64_t piece = std::max<int64_t>(1, units / (4 * gmax));  // cost per item
    int64_t slots[BATCH_CLASSES] = {0, 0};
    for (int s = 0; s < batch; ++s) {
        const SeriesDesc &d = sd[s];
        for (int R = 0; R < d.TR; ++R)
            for (int Cc = 0; Cc <= R; ++Cc) {
                const int ct = chunk_cost(d.cls, Cc == R);
                const int64_t pc = std::max<int64_t>(1, piece / ct);
                C3TileRef t;
                t.series = s;
                t.R = R;
                t.Cc = Cc;
                t.slot0 = slots[d.cls];
                t.nslot = 0;
                for (int64_t c0 = 0; c0 < d.C; c0 += pc) {
                    C3Item it;
                    it.series = s;
                    it.R = R;
                    it.Cc = Cc;
                    it.pad = d.cls;
                    it.c0 = c0;
                    it.c1 = std::min<int64_t>(d.C, c0 + pc);
                    it.slot = slots[d.cls]++;
                    items.push_back(it);
                    cost.push_back((it.c1 - it.c0) * ct);
                    t.nslot++;
                    h.n_items[d.cls]++;
                }
                tiles[d.cls].push_back(t);
            }
    }
    const int64_t ni = (int64_t)items.size();
    const int64_t G = std::min<int64_t>(gmax, ni);
    if (ni > 0) {
        // longest processing time first, ties in plan order
        std::vector<int64_t> ord(ni);
        for (int64_t k = 0; k < ni; ++k)
            ord[k] = k;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
        typedef std::pair<int64_t, int64_t> LW;   // (load, workgroup)
        std::priority_queue<LW, std::vector<LW>, std::greater<LW>> heap;
        for (int64_t w = 0; w < G; ++w)
            heap.push(LW(0, w));
        std::vector<std::vector<int64_t>> per(G);
        for (int64_t k : ord) {
            LW top = heap.top();
            heap.pop();
            per[top.second].push_back(k);
            heap.push(LW(top.first + cost[k], top.second));
        }
        std::vector<C3Item> sorted;
        sorted.reserve(ni);
        wgfirst.push_back(0);
        for (int64_t w = 0; w < G; ++w) {
            // the kernel runs a workgroup's 4 x 4-block items first, then its
            // 2 x 2-block items (one loop per class)
            for (int cls = 1; cls >= 0; --cls)
                for (int64_t k : per[w])
                    if (items[k].pad == cls)
                        sorted.push_back(items[k]);
            wgfirst.push_back((int32_t)sorted.size());
        }
        items.swap(sorted);
    }
    h.n_items_all = ni;
    for (int cls = 0; cls < BATCH_CLASSES; ++cls) {
        h.G[cls] = G;
        h.n_tiles[cls] = (int64_t)tiles[cls].size();
        const int64_t tile = (int64_t)(32 * (cls ? 4 : 2)) * (32 * (cls ? 4 : 2));
        h.part_off[cls] = (int64_t)o;
        o = a256(o + (size_t)slots[cls] * tile * sizeof(double));
    }
    h.ws_bytes = (int64_t)o;

    // blob: header | series | items | wgfirst | tiles per class | groups
    size_t b = up(sizeof(BatchHeader), 64);
    h.series_off = (int64_t)b;
    b += sizeof(SeriesDesc) * batch;
    h.items_off = (int64_t)b;
    b += sizeof(C3Item) * items.size();
    h.wgfirst_off = (int64_t)b;
    b += up(sizeof(int32_t) * wgfirst.size(), 8);
    for (int cls = 0; cls < BATCH_CLASSES; ++cls) {
        h.tiles_off[cls] = (int64_t)b;
        b += sizeof(C3TileRef) * tiles[cls].size();
    }
    h.groups_off = (int64_t)b;
    h.n_groups = (int64_t)groups.size();
    b += sizeof(FftGroup) * groups.size();
    h.gseries_off = (int64_t)b;
    b += up(sizeof(int32_t) * batch, 8);
    h.blob_bytes = (int64_t)up(b, 256);

    if (hdr_out)
        *hdr_out = h;
    if (!blob)
        return HOS_OK;
    if (blob_bytes < (size_t)h.blob_bytes)
        return HOS_EINVAL;
    char *p = (char *)blob;
    memset(p, 0, h.blob_bytes);
    memcpy(p, &h, sizeof(h));
    memcpy(p + h.series_off, sd.data(), sizeof(SeriesDesc) * batch);
    if (!items.empty())
        memcpy(p + h.items_off, items.data(), sizeof(C3Item) * items.size());
    if (!wgfirst.empty())
        memcpy(p + h.wgfirst_off, wgfirst.data(), sizeof(int32_t) * wgfirst.size());
    for (int cls = 0; cls < BATCH_CLASSES; ++cls)
        if (!tiles[cls].empty())
            memcpy(p + h.tiles_off[cls], tiles[cls].data(), sizeof(C3TileRef) * tiles[cls].size());
    memcpy(p + h.groups_off, groups.data(), sizeof(FftGroup) * groups.size());
    memcpy(p + h.gseries_off, gseries.data(), sizeof(int32_t) * batch);
    return HOS_OK;
}

// The host copy of a plan, checked for integrity.
static const BatchHeader *plan_header(const void *plan_host)
{
    if (!plan_host || ((uintptr_t)plan_host & 7))
        return nullptr;
    const BatchHeader *h = (const BatchHeader *)plan_host;
    if (h->magic != BATCH_MAGIC || h->batch < 1 || h->blob_bytes < (int64_t)sizeof(BatchHeader))
        return nullptr;
    return h;
}

static bool aligned_to(const void *p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace hos

using namespace hos;

extern "C" {

int hos_batch_plan_size(int32_t batch, const int64_t *n, const int32_t *M, int32_t window,
                        int32_t path, uint32_t flags, const int32_t *tile_nb, size_t *plan_bytes,
                        size_t *ws_bytes)
{
    if (!plan_bytes || !ws_bytes)
        return HOS_EINVAL;
    BatchHeader h;
    const int st = batch_plan(batch, n, M, window, path, flags, tile_nb, nullptr, 0, &h);
    if (st != HOS_OK)
        return st;
    *plan_bytes = (size_t)h.blob_bytes;
    *ws_bytes = (size_t)h.ws_bytes;
    return HOS_OK;
}

int hos_batch_plan(int32_t batch, const int64_t *n, const int32_t *M, int32_t window,
                   int32_t path, uint32_t flags, const int32_t *tile_nb, void *plan,
                   size_t plan_bytes)
{
    if (!plan || !aligned_to(plan, 8))
        return HOS_EINVAL;
    return batch_plan(batch, n, M, window, path, flags, tile_nb, plan, plan_bytes, nullptr);
}

int hos_batch_plan_info(const void *plan, int64_t *info, int32_t ninfo)
{
    const BatchHeader *h = plan_header(plan);
    if (!h || !info || ninfo < 12)
        return HOS_EINVAL;
    info[0] = h->batch;
    info[1] = h->c3_total;
    info[2] = h->pd_total;
    info[3] = h->x_total;
    info[4] = h->ws_bytes;
    info[5] = h->blob_bytes;
    info[6] = h->n_items[0];
    info[7] = h->n_items[1];
    info[8] = h->G[0];
    info[9] = h->G[1];
    info[10] = h->uniform_M;
    info[11] = h->max_npd;
    return HOS_OK;
}

// Host-only listing of the plan's work items, for tests: row k of `out`
// (7 int64 each) = class, workgroup, series, R, Cc, c0, c1 ... plus slot.
int hos_batch_items(const void *plan, int32_t cls, int64_t *out, int64_t cap)
{
    const BatchHeader *h = plan_header(plan);
    if (!h || !out || cls < -1 || cls >= BATCH_CLASSES)
        return HOS_EINVAL;
    const int64_t ni = cls < 0 ? h->n_items_all : h->n_items[cls];
    if (cap < ni * 8)
        return HOS_EINVAL;
    if (h->n_items_all == 0)
        return HOS_OK;
    const char *p = (const char *)plan;
    const C3Item *it = (const C3Item *)(p + h->items_off);
    const int32_t *wf = (const int32_t *)(p + h->wgfirst_off);
    int64_t row = 0;
    for (int64_t w = 0; w < h->G[0]; ++w)
        for (int64_t k = wf[w]; k < wf[w + 1]; ++k) {
            if (cls >= 0 && it[k].pad != cls)
                continue;
            int64_t *r = out + 8 * row++;
            r[0] = it[k].pad;
            r[1] = w;
            r[2] = it[k].series;
            r[3] = it[k].R;
            r[4] = it[k].Cc;
            r[5] = it[k].c0;
            r[6] = it[k].c1;
            r[7] = it[k].slot;
        }
    return HOS_OK;
}

// Per-series layout for tests: row s (8 int64) = n, M, N, npd, x_off, c3_off,
// pd_off, cls.
int hos_batch_series(const void *plan, int64_t *out, int64_t cap)
{
    const BatchHeader *h = plan_header(plan);
    if (!h || !out || cap < h->batch * 8)
        return HOS_EINVAL;
    const SeriesDesc *sd = (const SeriesDesc *)((const char *)plan + h->series_off);
    for (int64_t s = 0; s < h->batch; ++s) {
        int64_t *r = out + 8 * s;
        r[0] = sd[s].n;
        r[1] = sd[s].M;
        r[2] = sd[s].N;
        r[3] = sd[s].npd;
        r[4] = sd[s].x_off;
        r[5] = sd[s].c3_off;
        r[6] = sd[s].pd_off;
        r[7] = sd[s].cls;
    }
    return HOS_OK;
}

static int batch_common(const void *x, int32_t dtype, const void *plan_host,
                        const void *plan_dev, void *ws, size_t ws_bytes,
                        const BatchHeader **hout)
{
    const BatchHeader *h = plan_header(plan_host);
    if (!h || !x || !plan_dev || !ws)
        return HOS_EINVAL;
    if (dtype != HOS_F32 && dtype != HOS_F64)
        return HOS_EINVAL;
    if (!aligned_to(x, dtype == HOS_F64 ? 8 : 4) || !aligned_to(ws, 256) ||
        !aligned_to(plan_dev, 256))
        return HOS_EINVAL;
    if (ws_bytes < (size_t)h->ws_bytes)
        return HOS_EWORKSPACE;
    *hout = h;
    return device_ok_public();
}

// The shared forward: moments, operands, contraction, reduction.
static hipError_t batch_forward(const void *x, int32_t dtype, const BatchHeader &h,
                                const char *dplan, char *w, hipStream_t stream)
{
    hipError_t e = launch_batch_prep(x, dtype, h, dplan, w, stream);
    if (e == hipSuccess) e = launch_batch_contract(h, dplan, w, stream);
    if (e == hipSuccess) e = launch_batch_reduce(x, dtype, h, dplan, w, stream);
    return e;
}

static int batched_impl(const void *x, int32_t dtype, const void *plan_host,
                        const void *plan_dev, double *c3, double *B_pd, void *ws,
                        size_t ws_bytes, hipStream_t stream, hipEvent_t *ev)
{
    const BatchHeader *h = nullptr;
    if (!c3 && !B_pd)
        return HOS_EINVAL;
    if ((c3 && !aligned_to(c3, 8)) || (B_pd && !aligned_to(B_pd, 16)))
        return HOS_EINVAL;
    int st = batch_common(x, dtype, plan_host, plan_dev, ws, ws_bytes, &h);
    if (st != HOS_OK)
        return st;
    char *w = (char *)ws;
    const char *dp = (const char *)plan_dev;
    auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], stream) : hipSuccess; };
    hipError_t e = mark(0);
    if (e == hipSuccess) e = launch_batch_prep(x, dtype, *h, dp, w, stream);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess) e = launch_batch_contract(*h, dp, w, stream);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = launch_batch_reduce(x, dtype, *h, dp, w, stream);
    if (e == hipSuccess) e = mark(3);
    if (e == hipSuccess) e = launch_batch_spectra(*h, dp, (int)h->window, c3, B_pd, w, stream);
    if (e == hipSuccess) e = mark(4);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

int hos_bispectrum_batched(const void *x, int32_t dtype, const void *plan_host,
                           const void *plan_dev, double *c3, double *B_pd, void *ws,
                           size_t ws_bytes, hipStream_t stream)
{
    return batched_impl(x, dtype, plan_host, plan_dev, c3, B_pd, ws, ws_bytes, stream, nullptr);
}

int hos_bispectrum_batched_timed(const void *x, int32_t dtype, const void *plan_host,
                                 const void *plan_dev, double *c3, double *B_pd, void *ws,
                                 size_t ws_bytes, hipStream_t stream, float *stage_ms)
{
    if (!stage_ms)
        return HOS_EINVAL;
    hipEvent_t ev[5];
    int made = 0;
    for (; made < 5; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess)
            break;
    int st = made == 5 ? batched_impl(x, dtype, plan_host, plan_dev, c3, B_pd, ws, ws_bytes,
                                      stream, ev)
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

int hos_bispectrum_segments(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, double *c3, double *B, void *ws,
                            size_t ws_bytes, hipStream_t stream)
{
    if (!c3 && !B)
        return HOS_EINVAL;
    if ((c3 && !aligned_to(c3, 8)) || (B && !aligned_to(B, 16)))
        return HOS_EINVAL;
    const BatchHeader *hh = plan_header(plan_host);
    if (hh && (hh->uniform_M < 0 || !(hh->flags & HOS_PLAN_SEGMENTS)))
        return HOS_EINVAL;
    const BatchHeader *h = nullptr;
    int st = batch_common(x, dtype, plan_host, plan_dev, ws, ws_bytes, &h);
    if (st != HOS_OK)
        return st;
    char *w = (char *)ws;
    const char *dp = (const char *)plan_dev;
    const SeriesDesc *sd = (const SeriesDesc *)((const char *)plan_host + h->series_off);
    const int M = (int)h->uniform_M, N = sd[0].N;
    const int64_t ne = (int64_t)(M + 1) * (M + 1);
    const double *avg = (const double *)(w + h->seg_off);
    double2 *tw = (double2 *)(w + h->seg_off + a256((size_t)(ne + 64) * sizeof(double)));
    hipError_t e = batch_forward(x, dtype, *h, dp, w, stream);
    if (e == hipSuccess) e = launch_seg_average(*h, dp, w, stream);
    if (e == hipSuccess && B) e = launch_twiddles(tw, N, stream);
    if (e == hipSuccess)
        e = launch_c3_finish_table(avg, avg + ne, M, M, (int)h->window, N, tw, c3, M, B,
                                   stream);
    if (e == hipSuccess && B) e = launch_fft_cols(B, N, tw, stream);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

int hos_bispectrum_loss_fwd(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, const double *target_pd, double *B_pd,
                            double *loss, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const BatchHeader *h = nullptr;
    if (!target_pd || !B_pd || !loss)
        return HOS_EINVAL;
    if (!aligned_to(target_pd, 16) || !aligned_to(B_pd, 16) || !aligned_to(loss, 8))
        return HOS_EINVAL;
    const BatchHeader *hh = plan_header(plan_host);
    if (hh && hh->uniform_M < 0)
        return HOS_EINVAL;   // one target needs one DFT size
    int st = batch_common(x, dtype, plan_host, plan_dev, ws, ws_bytes, &h);
    if (st != HOS_OK)
        return st;
    char *w = (char *)ws;
    hipError_t e = batch_forward(x, dtype, *h, (const char *)plan_dev, w, stream);
    if (e == hipSuccess)
        e = launch_batch_spectra(*h, (const char *)plan_dev, (int)h->window, nullptr, B_pd, w,
                                 stream);
    if (e == hipSuccess)
        e = launch_batch_loss(*h, (const char *)plan_dev, B_pd, target_pd, loss, w, stream);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

int hos_bispectrum_loss_bwd(const void *x, int32_t dtype, const void *plan_host,
                            const void *plan_dev, const double *B_pd, const double *target_pd,
                            const double *dL, void *dx, void *ws, size_t ws_bytes,
                            hipStream_t stream)
{
    const BatchHeader *h = nullptr;
    if (!B_pd || !target_pd || !dL || !dx)
        return HOS_EINVAL;
    if (!aligned_to(B_pd, 16) || !aligned_to(target_pd, 16) || !aligned_to(dL, 8) ||
        !aligned_to(dx, dtype == HOS_F64 ? 8 : 4))
        return HOS_EINVAL;
    const BatchHeader *hh = plan_header(plan_host);
    if (hh && (hh->uniform_M < 0 || !(hh->flags & HOS_PLAN_ADJOINT)))
        return HOS_EINVAL;
    int st = batch_common(x, dtype, plan_host, plan_dev, ws, ws_bytes, &h);
    if (st != HOS_OK)
        return st;
    char *w = (char *)ws;
    hipError_t e = launch_batch_prep(x, dtype, *h, (const char *)plan_dev, w, stream);
    if (e == hipSuccess)
        e = launch_batch_adjoint(x, dtype, *h, (const char *)plan_dev, (int)h->window, B_pd,
                                 target_pd, dL, dx, w, stream);
    return e == hipSuccess ? HOS_OK : HOS_EDEVICE;
}

}  // extern "C"
