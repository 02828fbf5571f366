// api.cpp — the C ABI of libtumordb (argument checks, workspace layout, launch order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/tumornn.h"
#include "internal.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(DB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool live(const db_t *db) { return db && db->magic == tdb::kMagic; }

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

namespace tdb {

int tdb_set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

bool tdb_live(const db_t *db) { return live(db); }

bool make_geometry(int nx, int ny, int nz, Geometry *g)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 32 != 0)
        return false;
    const int64_t V = (int64_t)nx * ny * nz;
    // Word indices are int32 and the batched kernel divides row numbers by
    // ny with a 32-bit reciprocal: keep ny * ny * nz below 2^32.
    if (V / 32 >= (int64_t)1 << 27 || (int64_t)ny * ny * nz >= ((int64_t)1 << 32))
        return false;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->V = V;
    g->W = (int)(V / 32);
    g->Wp = (int)align_up((size_t)g->W, 4);
    g->nxw = nx / 32;
    return true;
}

WsLayout ws_layout(const db_t *db, int nq, int k, bool batched)
{
    WsLayout L{};
    const int64_t cap = db->capacity;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    L.qpack = take((size_t)nq * 2 * db->g.Wp * 4);
    L.qpart = take((size_t)nq * kQueryParts * sizeof(QueryPart));
    L.acnt = take((size_t)nq * 2 * 4);
    L.rois = take((size_t)nq * 6 * 4);
    L.qbox = take((size_t)nq * 4 * 4);
    L.qtbox = take((size_t)nq * 4 * 4);
    L.qmom = take((size_t)nq * 4 * 8);
    L.inter = take((size_t)nq * cap * 2 * 4);
    L.bcnt = batched ? take((size_t)nq * cap * 2 * 4) : off;
    // plan: query order [nq], 8 queue counters, slab list offsets [nq * nz + 1] and
    // slab lists [nq * nz] (at most one chunk per query and one slab per plane)
    L.plan = take(((size_t)nq + 8 + 2 * (size_t)nq * db->g.nz + 1) * 4);
    const size_t cand = (size_t)nq * topk_blocks(cap) * k;
    L.topk_a = take(cand * 12);
    L.topk_b = take(cand * 12);
    L.total = off;
    return L;
}

// Host state of a cached batched-query graph.
struct BatchGraph {
    int nq = 0, k = 0, Z = 0, threads = 0, tile = 0, qchunk = 0;
    int64_t n = 0;
    const void *labels = nullptr, *ws = nullptr, *idx = nullptr, *score = nullptr,
               *counts = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *staging = nullptr;  // pinned upload buffer: rois [nq][6] + order [nq]
    size_t staging_elems = 0;
    hipEvent_t uploaded = nullptr;
    bool upload_pending = false;

    void drop_exec()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    ~BatchGraph()
    {
        drop_exec();
        if (uploaded) {
            if (upload_pending) (void)hipEventSynchronize(uploaded);
            (void)hipEventDestroy(uploaded);
        }
        if (staging) (void)hipHostFree(staging);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Event pairs recorded around each launch of the dominant kernel (the scan,
// or the whole batched graph) while profiling is on.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;  // start, stop, start, stop, ...
    size_t used = 0;             // events recorded since the last read

    hipError_t mark(hipStream_t s)
    {
        if (used == ev.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        return hipEventRecord(ev[used++], s);
    }
    ~Profiler()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

}  // namespace tdb

using namespace tdb;

// Start/stop marks around the dominant kernel when profiling is on.
static hipError_t prof_mark(const db_t *db, hipStream_t s)
{
    if (!db->prof || !db->prof->on) return hipSuccess;
    return db->prof->mark(s);
}


static int check_query_common(const char *fn, const db_t *db, const uint8_t *q_labels, void *ws)
{
    if (!live(db)) return fail(DB_ESTATE, "%s: invalid handle", fn);
    if (db->count <= 0) return fail(DB_EINVAL, "%s: database is empty", fn);
    if (!q_labels || !aligned(q_labels, 16))
        return fail(DB_EINVAL, "%s: q_labels must be non-NULL and 16-byte aligned", fn);
    if (!ws || !aligned(ws, kAlign))
        return fail(DB_EINVAL, "%s: workspace must be non-NULL and 256-byte aligned", fn);
    return DB_OK;
}

template <class T>
static T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Enqueue the kernel sequence of a batched query on stream s.
static hipError_t enqueue_batch(const db_t *db, int nq, const uint8_t *q_labels, int k,
                                int32_t *idx, double *score, db_counts_t *counts, void *ws,
                                const WsLayout &L, const BatchPlan &P, hipStream_t s)
{
    uint32_t *qpack = at<uint32_t>(ws, L.qpack);
    uint32_t *acnt = at<uint32_t>(ws, L.acnt);
    uint32_t *inter = at<uint32_t>(ws, L.inter);
    uint32_t *bcnt = at<uint32_t>(ws, L.bcnt);
    int32_t *rois = at<int32_t>(ws, L.rois);
    int32_t *order = at<int32_t>(ws, L.plan);
    int32_t *counters = order + nq;
    int32_t *list_off = counters + 8;
    int32_t *list_q = list_off + (size_t)nq * db->g.nz + 1;
    QueryPart *qpart = at<QueryPart>(ws, L.qpart);
    hipError_t e = launch_pack_queries(db, q_labels, nq, rois, qpack, qpart, s);
    if (e == hipSuccess)
        e = launch_sum_parts(qpart, nq, acnt, at<int32_t>(ws, L.qbox), at<uint64_t>(ws, L.qmom), s);
    if (e == hipSuccess) e = launch_fill_u32(counters, 8, 0, s);
    if (e == hipSuccess)
        e = launch_batch_scan(db, db->count, nq, P, qpack, rois, order, list_off, list_q, counters,
                              inter, bcnt, s);
    if (e == hipSuccess) {
        TopkArgs a{};
        a.n = db->count;
        a.nq = nq;
        a.k = k;
        a.inter = inter;
        a.inter_qstride = 2 * db->capacity;
        a.bcnt = bcnt;
        a.bcnt_qstride = 2 * db->capacity;
        a.acnt = acnt;
        const size_t cand = (size_t)nq * topk_blocks(db->capacity) * k;
        a.buf_s[0] = at<uint64_t>(ws, L.topk_a);
        a.buf_s[1] = at<uint64_t>(ws, L.topk_b);
        a.buf_i[0] = reinterpret_cast<int32_t *>(a.buf_s[0] + cand);
        a.buf_i[1] = reinterpret_cast<int32_t *>(a.buf_s[1] + cand);
        a.out_idx = idx;
        a.out_score = score;
        a.out_counts = counts;
        e = launch_topk(a, s);
    }
    return e;
}

// Argument checks of a distance launch (nothing is enqueued).
static int dist_check(const char *fn, int fmt, int M, int N, int dim, const void *q_codes,
                      const float *q_scale, const float *q_sq, const void *x_codes,
                      const float *x_scale, const float *x_sq, const float *D)
{
    if (M <= 0 || N <= 0 || dim <= 0 || !q_codes || !x_codes || !D || (M + 127) / 128 > 65535)
        return fail(DB_EINVAL, "%s: bad arguments", fn);
    if (fmt != EMB_BIN && (!q_sq || !x_sq))
        return fail(DB_EINVAL, "%s: squared norms are required", fn);
    if (fmt != EMB_BIN && (int64_t)M * dim * (fmt == EMB_BF16 ? 2 : 1) >= ((int64_t)1 << 31))
        return fail(DB_EINVAL, "%s: query codes must stay below 2 GiB", fn);
    if (fmt == EMB_BIN) {
        if (dim % 32 || dim > 1024)
            return fail(DB_EINVAL, "%s: binary codes need dim %% 32 == 0, <= 1024", fn);
    } else if (fmt == EMB_BF16) {
        if (dim % 16) return fail(DB_EINVAL, "%s: BF16 needs dim %% 16 == 0", fn);
        if (!aligned(q_codes, 16) || !aligned(x_codes, 16))
            return fail(DB_EINVAL, "%s: codes must be 16-byte aligned", fn);
    } else if (fmt == EMB_FP8) {
        if (dim % 64 || !q_scale || !x_scale)
            return fail(DB_EINVAL, "%s: FP8 needs dim %% 64 == 0 and scales", fn);
        if (!aligned(q_codes, 32) || !aligned(x_codes, 32))
            return fail(DB_EINVAL, "%s: codes must be 32-byte aligned", fn);
    } else {
        return fail(DB_EINVAL, "%s: unknown format %d", fn, fmt);
    }
    return DB_OK;
}

static hipError_t dist_launch(int fmt, int M, int N, int dim, const void *q_codes,
                              const float *q_scale, const float *q_sq, const void *x_codes,
                              const float *x_scale, const float *x_sq, float *D, int mode,
                              hipStream_t s, uint32_t *gmin = nullptr)
{
    if (fmt == EMB_BIN)
        return launch_hamming(M, N, dim / 32, static_cast<const uint32_t *>(q_codes),
                              static_cast<const uint32_t *>(x_codes), D, s);
    if (fmt == EMB_BF16)
        return launch_dist_bf16(M, N, dim, static_cast<const uint16_t *>(q_codes), q_sq,
                                static_cast<const uint16_t *>(x_codes), x_sq, D, mode, gmin, s);
    return launch_dist_fp8(M, N, dim, static_cast<const uint8_t *>(q_codes), q_scale, q_sq,
                           static_cast<const uint8_t *>(x_codes), x_scale, x_sq, D, mode, gmin, s);
}

// Sort the entries by the centre of their row boxes (z in bands of 8 planes,
// then y), so that the batched kernel's tiles (groups of `tile` consecutive
// entries) hold overlapping boxes; then order the tiles by the size of the union
// of their members' row boxes, largest first (blocks are dispatched in this
// order, so the longest items start first). Reads the boxes back after a
// device synchronisation; host sort; one upload.
static int build_tile_order(db_t *db, int tile)
{
    const int64_t n = db->count;
    std::vector<int32_t> box((size_t)n * 4);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(box.data(), db->box, (size_t)n * 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "db_query_batch: read row boxes");
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto empty = [&](int32_t i) {
        const int32_t *b = &box[(size_t)i * 4];
        return !(b[1] > b[0] && b[3] > b[2]);
    };
    auto key = [&](int32_t i) {
        const int32_t *b = &box[(size_t)i * 4];
        const int64_t zc = b[0] + b[1], yc = b[2] + b[3];
        return empty(i) ? INT64_MAX : ((zc / 16) << 32) | (yc << 16) | (b[1] - b[0]);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return key(a) < key(b); });
    const int64_t ntiles = (n + tile - 1) / tile;
    std::vector<int64_t> tcost(ntiles, 0);
    for (int64_t t = 0; t < ntiles; ++t) {
        int z0 = INT32_MAX, z1 = INT32_MIN, y0 = INT32_MAX, y1 = INT32_MIN;
        for (int64_t j = t * tile; j < std::min<int64_t>(n, (t + 1) * tile); ++j) {
            if (empty(order[j])) continue;
            const int32_t *b = &box[(size_t)order[j] * 4];
            z0 = std::min(z0, b[0]);
            z1 = std::max(z1, b[1]);
            y0 = std::min(y0, b[2]);
            y1 = std::max(y1, b[3]);
        }
        tcost[t] = z1 > z0 ? (int64_t)(z1 - z0) * (y1 - y0) : 0;
    }
    // The last (partial) tile keeps its place: tiles are read as groups of `tile` entries.
    std::vector<int64_t> tperm(ntiles);
    std::iota(tperm.begin(), tperm.end(), 0);
    const int64_t nfull = n / tile;
    std::stable_sort(tperm.begin(), tperm.begin() + nfull,
                     [&](int64_t a, int64_t b) { return tcost[a] > tcost[b]; });
    std::vector<int32_t> sorted;
    sorted.reserve(n);
    for (int64_t t : tperm)
        for (int64_t j = t * tile; j < std::min<int64_t>(n, (t + 1) * tile); ++j)
            sorted.push_back(order[j]);
    e = hipMemcpy(db->tile_order, sorted.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "db_query_batch: upload tile order");
    db->tile_order_n = n;
    db->tile_order_tile = tile;
    return DB_OK;
}

// Block counts of entry e (nullptr when the grid has too many blocks to keep them).
static uint16_t *block_counts_at(const db_t *db, int64_t e)
{
    return db->bcnt ? db->bcnt + e * 2 * bound_blocks(db->g, nullptr, nullptr) : nullptr;
}

extern "C" {

size_t db_storage_bytes(int nx, int ny, int nz, int64_t capacity)
{
    Geometry g;
    if (!make_geometry(nx, ny, nz, &g) || capacity <= 0 || capacity > INT32_MAX)
        return 0;
    const int nbp = bound_blocks(g, nullptr, nullptr);
    return align_up((size_t)capacity * 2 * g.Wp * 4, kAlign) +
           align_up((size_t)capacity * 2 * 4, kAlign) + align_up((size_t)capacity * 4 * 4, kAlign) +
           align_up((size_t)capacity * 4 * 8, kAlign) + align_up((size_t)capacity * 4, kAlign) +
           align_up((size_t)capacity * 4 * 4, kAlign) + align_up((size_t)capacity * nz * 2 * 4, kAlign) +
           align_up((size_t)capacity * 2 * nbp * 2, kAlign);
}

int db_build(db_t **out, int nx, int ny, int nz, float t_lo, float t_hi, int64_t capacity,
             void *storage, size_t storage_bytes)
{
    if (!out) return fail(DB_EINVAL, "db_build: out is NULL");
    Geometry g;
    if (!make_geometry(nx, ny, nz, &g))
        return fail(DB_EINVAL, "db_build: bad grid %dx%dx%d (need positive dims, nx %% 32 == 0)",
                    nx, ny, nz);
    if (capacity <= 0 || capacity > INT32_MAX)
        return fail(DB_EINVAL, "db_build: capacity %lld out of range", (long long)capacity);
    if (!(t_lo == t_lo) || !(t_hi == t_hi) || !(t_lo < t_hi))
        return fail(DB_EINVAL, "db_build: need t_lo < t_hi (got %g, %g)", t_lo, t_hi);
    if (!storage || !aligned(storage, kAlign))
        return fail(DB_EINVAL, "db_build: storage must be non-NULL and 256-byte aligned");
    const size_t need = db_storage_bytes(nx, ny, nz, capacity);
    if (storage_bytes < need)
        return fail(DB_ENOSPC, "db_build: storage %zu bytes < %zu needed", storage_bytes, need);
    int dev = 0, cus = 0, lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "db_build: device query");
    // Let the batched kernel use all of it (above the default dynamic limit).
    if (batch_set_lds_limit(lds) != hipSuccess) {
        (void)hipGetLastError();
        lds = 65536;
    }
    db_t *db = new (std::nothrow) db_t{};
    if (!db) return fail(DB_ENOMEM, "db_build: out of host memory");
    db->magic = kMagic;
    db->g = g;
    db->t_lo = t_lo;
    db->t_hi = t_hi;
    db->capacity = capacity;
    db->count = 0;
    db->planes = static_cast<uint32_t *>(storage);
    const size_t o_pc = align_up((size_t)capacity * 2 * g.Wp * 4, kAlign);
    const size_t o_box = o_pc + align_up((size_t)capacity * 2 * 4, kAlign);
    const size_t o_mom = o_box + align_up((size_t)capacity * 4 * 4, kAlign);
    db->popcnt = reinterpret_cast<uint32_t *>(static_cast<char *>(storage) + o_pc);
    db->box = reinterpret_cast<int32_t *>(static_cast<char *>(storage) + o_box);
    db->mom = reinterpret_cast<uint64_t *>(static_cast<char *>(storage) + o_mom);
    const size_t o_ord = o_mom + align_up((size_t)capacity * 4 * 8, kAlign);
    db->tile_order = reinterpret_cast<int32_t *>(static_cast<char *>(storage) + o_ord);
    const size_t o_tbox = o_ord + align_up((size_t)capacity * 4, kAlign);
    db->tbox = reinterpret_cast<int32_t *>(static_cast<char *>(storage) + o_tbox);
    const size_t o_zr = o_tbox + align_up((size_t)capacity * 4 * 4, kAlign);
    db->zrange = reinterpret_cast<uint32_t *>(static_cast<char *>(storage) + o_zr);
    const size_t o_bc = o_zr + align_up((size_t)capacity * nz * 2 * 4, kAlign);
    db->bcnt = bound_blocks(g, nullptr, nullptr)
                   ? reinterpret_cast<uint16_t *>(static_cast<char *>(storage) + o_bc)
                   : nullptr;
    db->rerank_bound = 1;
    db->tile_order_n = 0;
    db->storage_bytes = storage_bytes;
    db->cus = cus;
    db->device = dev;
    db->lds_max = lds;
    db->batch_planes = 0;
    db->batch_threads = 0;
    db->batch_tile = 0;
    db->batch_qchunk = 0;
    db->tile_order_tile = 0;
    db->graph = nullptr;
    db->prof = nullptr;
    *out = db;
    g_err[0] = 0;
    return DB_OK;
}

int db_append(db_t *db, const float *conc, int64_t n, void *stream)
{
    if (!live(db)) return fail(DB_ESTATE, "db_append: invalid handle");
    if (n < 0) return fail(DB_EINVAL, "db_append: n < 0");
    if (n == 0) return DB_OK;
    if (!conc || !aligned(conc, 16))
        return fail(DB_EINVAL, "db_append: conc must be non-NULL and 16-byte aligned");
    if (db->count + n > db->capacity)
        return fail(DB_ENOSPC, "db_append: %lld + %lld entries exceed capacity %lld",
                    (long long)db->count, (long long)n, (long long)db->capacity);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *planes = db->planes + db->count * 2 * (int64_t)db->g.Wp;
    uint32_t *pc = db->popcnt + db->count * 2;
    hipError_t e = launch_pack_db(db, conc, n, planes, pc, s);
    if (e == hipSuccess)
        e = launch_meta(planes, n, db->g, db->box + db->count * 4, db->tbox + db->count * 4,
                        db->mom + db->count * 4, db->zrange + db->count * db->g.nz * 2, s);
    if (e == hipSuccess)
        e = launch_block_counts(db, planes, n, db->box + db->count * 4, block_counts_at(db, db->count),
                                s);
    if (e != hipSuccess) return hip_fail(e, "db_append: launch");
    db->count += n;
    return DB_OK;
}

int64_t db_size(const db_t *db) { return live(db) ? db->count : -1; }

size_t db_query_workspace_bytes(const db_t *db, int nq, int k)
{
    if (!live(db) || nq <= 0 || k <= 0 || k > DB_KMAX) return 0;
    return ws_layout(db, nq, k, true).total;
}

int db_scan(const db_t *db, const uint8_t *q_labels, uint32_t *inter, uint32_t *qcount, void *ws,
            size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_scan", db, q_labels, ws);
    if (rc) return rc;
    if (!inter) return fail(DB_EINVAL, "db_scan: inter is NULL");
    const WsLayout L = ws_layout(db, 1, 1, true);
    if (ws_bytes < L.total)
        return fail(DB_ENOSPC, "db_scan: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    QueryPart *qpart = at<QueryPart>(ws, L.qpart);
    hipError_t e = launch_pack_queries(db, q_labels, 1, nullptr, at<uint32_t>(ws, L.qpack), qpart, s);
    if (e == hipSuccess)
        e = launch_sum_parts(qpart, 1, qcount ? qcount : at<uint32_t>(ws, L.acnt),
                             at<int32_t>(ws, L.qbox), at<uint64_t>(ws, L.qmom), s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) e = launch_scan(db, db->count, at<uint32_t>(ws, L.qpack), inter, s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e != hipSuccess) return hip_fail(e, "db_scan: launch");
    return DB_OK;
}

}  // extern "C"

namespace tdb {

// The launches of one exact query (pack, scan, Dice + top-k) into ws laid out as L.
hipError_t enqueue_query(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx,
                         double *score, db_counts_t *counts, void *ws, const WsLayout &L,
                         hipStream_t s)
{
    uint32_t *inter = at<uint32_t>(ws, L.inter);
    uint32_t *acnt = at<uint32_t>(ws, L.acnt);
    QueryPart *qpart = at<QueryPart>(ws, L.qpart);
    hipError_t e = launch_pack_queries(db, q_labels, 1, nullptr, at<uint32_t>(ws, L.qpack), qpart, s);
    if (e == hipSuccess)
        e = launch_sum_parts(qpart, 1, acnt, at<int32_t>(ws, L.qbox), at<uint64_t>(ws, L.qmom), s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) e = launch_scan(db, db->count, at<uint32_t>(ws, L.qpack), inter, s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) {
        TopkArgs a{};
        a.n = db->count;
        a.nq = 1;
        a.k = k;
        a.inter = inter;
        a.inter_qstride = 0;
        a.bcnt = db->popcnt;
        a.bcnt_qstride = 0;
        a.acnt = acnt;
        a.buf_s[0] = at<uint64_t>(ws, L.topk_a);
        a.buf_s[1] = at<uint64_t>(ws, L.topk_b);
        const size_t cand = topk_blocks(db->capacity) * (size_t)k;
        a.buf_i[0] = reinterpret_cast<int32_t *>(a.buf_s[0] + cand);
        a.buf_i[1] = reinterpret_cast<int32_t *>(a.buf_s[1] + cand);
        a.out_idx = idx;
        a.out_score = score;
        a.out_counts = counts;
        e = launch_topk(a, s);
    }
    return e;
}

// Argument checks of a single exact query (everything but the workspace size).
int check_query_args(const char *fn, const db_t *db, const uint8_t *q_labels, int k,
                     const int32_t *idx, const double *score)
{
    if (!live(db)) return fail(DB_ESTATE, "%s: invalid handle", fn);
    if (db->count <= 0) return fail(DB_EINVAL, "%s: database is empty", fn);
    if (!q_labels || !aligned(q_labels, 16))
        return fail(DB_EINVAL, "%s: q_labels must be non-NULL and 16-byte aligned", fn);
    if (k < 1 || k > DB_KMAX || k > db->count)
        return fail(DB_EINVAL, "%s: k = %d outside [1, min(%lld, %d)]", fn, k,
                    (long long)db->count, DB_KMAX);
    if (!idx || !score) return fail(DB_EINVAL, "%s: idx and score must be non-NULL", fn);
    return DB_OK;
}

}  // namespace tdb

extern "C" {

int db_query(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx, double *score,
             db_counts_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_query", db, q_labels, ws);
    if (rc) return rc;
    rc = check_query_args("db_query", db, q_labels, k, idx, score);
    if (rc) return rc;
    const WsLayout L = ws_layout(db, 1, k, true);
    if (ws_bytes < L.total)
        return fail(DB_ENOSPC, "db_query: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    hipError_t e = enqueue_query(db, q_labels, k, idx, score, counts, ws, L,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "db_query: launch");
    return DB_OK;
}

int db_query_sparse(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx, double *score,
                    db_counts_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_query_sparse", db, q_labels, ws);
    if (rc) return rc;
    if (k < 1 || k > DB_KMAX || k > db->count)
        return fail(DB_EINVAL, "db_query_sparse: k = %d outside [1, min(%lld, %d)]", k,
                    (long long)db->count, DB_KMAX);
    if (!idx || !score) return fail(DB_EINVAL, "db_query_sparse: idx and score must be non-NULL");
    const WsLayout L = ws_layout(db, 1, k, true);
    if (ws_bytes < L.total)
        return fail(DB_ENOSPC, "db_query_sparse: workspace %zu bytes < %zu needed", ws_bytes,
                    L.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *qpack = at<uint32_t>(ws, L.qpack);
    uint32_t *inter = at<uint32_t>(ws, L.inter);
    uint32_t *acnt = at<uint32_t>(ws, L.acnt);
    int32_t *qbox = at<int32_t>(ws, L.qbox), *qtbox = at<int32_t>(ws, L.qtbox);
    QueryPart *qpart = at<QueryPart>(ws, L.qpart);
    hipError_t e = launch_pack_queries(db, q_labels, 1, nullptr, qpack, qpart, s);
    if (e == hipSuccess)
        e = launch_sum_parts(qpart, 1, acnt, qbox, at<uint64_t>(ws, L.qmom), s, qtbox);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) e = launch_box_scan(db, db->count, qpack, qbox, qtbox, inter, s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) {
        TopkArgs a{};
        a.n = db->count;
        a.nq = 1;
        a.k = k;
        a.inter = inter;
        a.inter_qstride = 0;
        a.bcnt = db->popcnt;
        a.bcnt_qstride = 0;
        a.acnt = acnt;
        a.buf_s[0] = at<uint64_t>(ws, L.topk_a);
        a.buf_s[1] = at<uint64_t>(ws, L.topk_b);
        const size_t cand = topk_blocks(db->capacity) * (size_t)k;
        a.buf_i[0] = reinterpret_cast<int32_t *>(a.buf_s[0] + cand);
        a.buf_i[1] = reinterpret_cast<int32_t *>(a.buf_s[1] + cand);
        a.out_idx = idx;
        a.out_score = score;
        a.out_counts = counts;
        e = launch_topk(a, s);
    }
    if (e != hipSuccess) return hip_fail(e, "db_query_sparse: launch");
    return DB_OK;
}

int db_query_batch(const db_t *db_c, int nq, const uint8_t *q_labels, const db_roi_t *rois, int k,
                   int32_t *idx, double *score, db_counts_t *counts, void *ws, size_t ws_bytes,
                   void *stream)
{
    int rc = check_query_common("db_query_batch", db_c, q_labels, ws);
    if (rc) return rc;
    db_t *db = const_cast<db_t *>(db_c);  // only the graph cache is mutated
    const Geometry &g = db->g;
    if (nq < 1) return fail(DB_EINVAL, "db_query_batch: nq = %d < 1", nq);
    if (k < 1 || k > DB_KMAX || k > db->count)
        return fail(DB_EINVAL, "db_query_batch: k = %d outside [1, min(%lld, %d)]", k,
                    (long long)db->count, DB_KMAX);
    if (!idx || !score) return fail(DB_EINVAL, "db_query_batch: idx and score must be non-NULL");
    const WsLayout L = ws_layout(db, nq, k, true);
    if (ws_bytes < L.total)
        return fail(DB_ENOSPC, "db_query_batch: workspace %zu bytes < %zu needed", ws_bytes,
                    L.total);
    // Boxes (host) -> validated copy + cost order of the queries.
    std::vector<int32_t> box((size_t)nq * 6);
    std::vector<int64_t> cost(nq);
    for (int q = 0; q < nq; ++q) {
        db_roi_t r = rois ? rois[q] : db_roi_t{0, 0, 0, g.nx, g.ny, g.nz};
        if (r.x0 < 0 || r.y0 < 0 || r.z0 < 0 || r.x1 > g.nx || r.y1 > g.ny || r.z1 > g.nz ||
            r.x0 >= r.x1 || r.y0 >= r.y1 || r.z0 >= r.z1)
            return fail(DB_EINVAL, "db_query_batch: ROI %d (%d,%d,%d)-(%d,%d,%d) is empty or "
                        "outside the %dx%dx%d grid", q, r.x0, r.y0, r.z0, r.x1, r.y1, r.z1,
                        g.nx, g.ny, g.nz);
        int32_t *b = &box[(size_t)q * 6];
        b[0] = r.x0; b[1] = r.y0; b[2] = r.z0; b[3] = r.x1; b[4] = r.y1; b[5] = r.z1;
        const int64_t nw = ((r.x1 - 1) >> 5) - (r.x0 >> 5) + 1;
        cost[q] = nw * (int64_t)(r.y1 - r.y0) * (r.z1 - r.z0);
    }
    std::vector<int32_t> order(nq);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    // Per (query chunk, z-slab): the queries whose box meets the slab, costliest first.
    const BatchPlan P = batch_plan(db, nq);
    std::vector<int32_t> list_off, list_q;
    if (P.use_lds) {
        list_off.reserve((size_t)P.nchunks * P.nslabs + 1);
        list_off.push_back(0);
        for (int c = 0; c < P.nchunks; ++c)
            for (int sl = 0; sl < P.nslabs; ++sl) {
                const int zs0 = sl * P.Z, zs1 = std::min(g.nz, zs0 + P.Z);
                for (int32_t q : order) {
                    if (q / P.qchunk != c) continue;
                    const int32_t *b = &box[(size_t)q * 6];
                    if (b[2] < zs1 && b[5] > zs0) list_q.push_back(q);
                }
                list_off.push_back((int32_t)list_q.size());
            }
    }

    // Entries grouped by row-box centre for the LDS kernel's tiles (rebuilt after appends).
    if (P.use_lds && (db->tile_order_n != db->count || db->tile_order_tile != P.tile)) {
        rc = build_tile_order(db, P.tile);
        if (rc) return rc;
    }
    if (!db->graph) {
        db->graph = new (std::nothrow) BatchGraph();
        if (!db->graph) return fail(DB_ENOMEM, "db_query_batch: out of host memory");
    }
    BatchGraph &G = *db->graph;
    hipError_t e = hipSuccess;
    if (!G.cap) {
        e = hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&G.uploaded, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "db_query_batch: stream/event create");
    }
    // Pinned staging buffer; wait for the previous upload before reusing it.
    const size_t elems = (size_t)nq * 7 + list_off.size() + list_q.size();
    if (G.upload_pending) {
        e = hipEventSynchronize(G.uploaded);
        if (e != hipSuccess) return hip_fail(e, "db_query_batch: wait for previous upload");
        G.upload_pending = false;
    }
    if (G.staging_elems < elems) {
        if (G.staging) (void)hipHostFree(G.staging);
        G.staging = nullptr;
        G.staging_elems = 0;
        e = hipHostMalloc((void **)&G.staging, elems * 4, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "db_query_batch: pinned staging");
        G.staging_elems = elems;
    }
    std::memcpy(G.staging, box.data(), (size_t)nq * 6 * 4);
    std::memcpy(G.staging + (size_t)nq * 6, order.data(), (size_t)nq * 4);
    int32_t *st_lists = G.staging + (size_t)nq * 7;
    if (!list_off.empty()) std::memcpy(st_lists, list_off.data(), list_off.size() * 4);
    if (!list_q.empty())
        std::memcpy(st_lists + list_off.size(), list_q.data(), list_q.size() * 4);

    // (Re)record the graph when the shape or any pointer changed.
    const bool same = G.exec && G.nq == nq && G.k == k && G.n == db->count && G.Z == P.Z &&
                      G.threads == P.threads && G.tile == P.tile && G.qchunk == P.qchunk &&
                      G.labels == q_labels && G.ws == ws && G.idx == idx && G.score == score &&
                      G.counts == counts;
    if (!same) {
        G.drop_exec();
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "db_query_batch: begin capture");
        hipError_t le = enqueue_batch(db, nq, q_labels, k, idx, score, counts, ws, L, P, G.cap);
        e = hipStreamEndCapture(G.cap, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "db_query_batch: record");
        }
        if (e != hipSuccess) return hip_fail(e, "db_query_batch: end capture");
        e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            G.exec = nullptr;
            return hip_fail(e, "db_query_batch: instantiate");
        }
        G.nq = nq;
        G.k = k;
        G.n = db->count;
        G.Z = P.Z;
        G.threads = P.threads;
        G.tile = P.tile;
        G.qchunk = P.qchunk;
        G.labels = q_labels;
        G.ws = ws;
        G.idx = idx;
        G.score = score;
        G.counts = counts;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(at<int32_t>(ws, L.rois), G.staging, (size_t)nq * 6 * 4,
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(at<int32_t>(ws, L.plan), G.staging + (size_t)nq * 6, (size_t)nq * 4,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !list_off.empty()) {
        int32_t *d_off = at<int32_t>(ws, L.plan) + nq + 8;
        int32_t *d_q = d_off + (size_t)nq * g.nz + 1;
        e = hipMemcpyAsync(d_off, st_lists, list_off.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !list_q.empty())
            e = hipMemcpyAsync(d_q, st_lists + list_off.size(), list_q.size() * 4,
                               hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipEventRecord(G.uploaded, s);
    if (e != hipSuccess) return hip_fail(e, "db_query_batch: upload");
    G.upload_pending = true;
    e = prof_mark(db, s);
    if (e == hipSuccess) e = hipGraphLaunch(G.exec, s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e != hipSuccess) return hip_fail(e, "db_query_batch: graph launch");
    return DB_OK;
}

// ---- embedding search ----

int emb_quantize(int64_t n, int dim, const float *lat, int fmt, void *codes, float *scale,
                 float *sqnorm, void *stream)
{
    if (n <= 0 || n > INT32_MAX || dim <= 0 || !lat || !codes || !sqnorm)
        return fail(DB_EINVAL, "emb_quantize: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (fmt == EMB_BF16) {
        if (dim % 16) return fail(DB_EINVAL, "emb_quantize: BF16 needs dim %% 16 == 0");
        e = launch_quant_bf16(n, dim, lat, static_cast<uint16_t *>(codes), sqnorm, s);
    } else if (fmt == EMB_FP8) {
        if (dim % 64 || !scale) return fail(DB_EINVAL, "emb_quantize: FP8 needs dim %% 64 == 0 and scale");
        e = launch_quant_fp8(n, dim, lat, static_cast<uint8_t *>(codes), scale, sqnorm, s);
    } else {
        return fail(DB_EINVAL, "emb_quantize: unknown format %d", fmt);
    }
    if (e != hipSuccess) return hip_fail(e, "emb_quantize: launch");
    return DB_OK;
}

int emb_distances(int fmt, int M, int N, int dim, const void *q_codes, const float *q_scale,
                  const float *q_sq, const void *x_codes, const float *x_scale, const float *x_sq,
                  float *D, void *stream)
{
    int rc = dist_check("emb_distances", fmt, M, N, dim, q_codes, q_scale, q_sq, x_codes, x_scale,
                        x_sq, D);
    if (rc) return rc;
    hipError_t e = dist_launch(fmt, M, N, dim, q_codes, q_scale, q_sq, x_codes, x_scale, x_sq, D,
                               0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_distances: launch");
    return DB_OK;
}

int emb_distances_l2sum(int fmt, int M, int N, int dim, const void *q1_codes,
                        const float *q1_scale, const float *q1_sq, const void *x1_codes,
                        const float *x1_scale, const float *x1_sq, const void *q2_codes,
                        const float *q2_scale, const float *q2_sq, const void *x2_codes,
                        const float *x2_scale, const float *x2_sq, float *D, void *stream)
{
    if (fmt == EMB_BIN) return fail(DB_EINVAL, "emb_distances_l2sum: BF16 or FP8 latents only");
    int rc = dist_check("emb_distances_l2sum", fmt, M, N, dim, q1_codes, q1_scale, q1_sq, x1_codes,
                        x1_scale, x1_sq, D);
    if (!rc)
        rc = dist_check("emb_distances_l2sum", fmt, M, N, dim, q2_codes, q2_scale, q2_sq, x2_codes,
                        x2_scale, x2_sq, D);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = dist_launch(fmt, M, N, dim, q1_codes, q1_scale, q1_sq, x1_codes, x1_scale, x1_sq,
                               D, 1, s);
    if (e == hipSuccess)
        e = dist_launch(fmt, M, N, dim, q2_codes, q2_scale, q2_sq, x2_codes, x2_scale, x2_sq, D, 2,
                        s);
    if (e != hipSuccess) return hip_fail(e, "emb_distances_l2sum: launch");
    return DB_OK;
}

int emb_hash_thresholds(int64_t n, int dim, const float *lat, float *thr, void *stream)
{
    if (n <= 0 || n > INT32_MAX || dim <= 0 || dim > 65535 || !lat || !thr)
        return fail(DB_EINVAL, "emb_hash_thresholds: bad arguments");
    hipError_t e = launch_col_kth(lat, n, dim, (n - 1) / 2, thr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_hash_thresholds: launch");
    return DB_OK;
}

int emb_binarize(int64_t n, int dim, const float *lat, const float *thr, uint32_t *codes,
                 void *stream)
{
    if (n <= 0 || dim <= 0 || dim % 32 || dim > 1024 || !lat || !thr || !codes ||
        !aligned(lat, 16) || !aligned(thr, 16))
        return fail(DB_EINVAL, "emb_binarize: bad arguments (dim %d; dim %% 32 == 0, <= 1024, "
                    "16-byte aligned inputs)", dim);
    hipError_t e = launch_binarize(lat, n, dim, thr, codes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_binarize: launch");
    return DB_OK;
}

int nn_bihalf_fwd(int dtype, int B, int D, const void *U, void *out, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || B > 4096 || D <= 0 || !U || !out)
        return fail(DB_EINVAL, "nn_bihalf_fwd: bad arguments");
    hipError_t e = launch_bihalf_fwd(dtype == NN_F64, B, D, U, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "nn_bihalf_fwd: launch");
    return DB_OK;
}

int nn_bihalf_bwd(int dtype, int B, int D, double gamma, const void *U, const void *Bc,
                  const void *G, void *dU, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || B > 4096 || D <= 0 || !U || !Bc ||
        !G || !dU)
        return fail(DB_EINVAL, "nn_bihalf_bwd: bad arguments");
    hipError_t e = launch_bihalf_bwd(dtype == NN_F64, B, D, gamma, U, Bc, G, dU,
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "nn_bihalf_bwd: launch");
    return DB_OK;
}

size_t emb_groups_workspace_bytes(int M, int N)
{
    if (M <= 0 || N <= 0) return 0;
    return topk_groups_ws_bytes(M, N);
}

int emb_distances_groups(int fmt, int M, int N, int dim, const void *q_codes,
                         const float *q_scale, const float *q_sq, const void *x_codes,
                         const float *x_scale, const float *x_sq, float *D, void *ws,
                         size_t ws_bytes, void *stream)
{
    int rc = dist_check("emb_distances_groups", fmt, M, N, dim, q_codes, q_scale, q_sq, x_codes,
                        x_scale, x_sq, D);
    if (rc) return rc;
    if (fmt == EMB_BIN) return fail(DB_EINVAL, "emb_distances_groups: BF16 or FP8 latents only");
    const size_t need = topk_groups_ws_bytes(M, N);
    if (!ws || !aligned(ws, 16) || ws_bytes < need)
        return fail(DB_ENOSPC, "emb_distances_groups: workspace %zu bytes < %zu needed (16-byte "
                    "aligned)", ws ? ws_bytes : 0, need);
    hipError_t e = dist_launch(fmt, M, N, dim, q_codes, q_scale, q_sq, x_codes, x_scale, x_sq, D,
                               0, static_cast<hipStream_t>(stream), topk_groups_gmin(ws, M));
    if (e != hipSuccess) return hip_fail(e, "emb_distances_groups: launch");
    return DB_OK;
}

int emb_topk_groups(int M, int N, const float *D, int k, int32_t *idx, float *d, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (M <= 0 || N <= 0 || !D || !idx || !d || k < 1 || k > N || k > DB_KMAX)
        return fail(DB_EINVAL, "emb_topk_groups: bad arguments (k = %d, N = %d)", k, N);
    const size_t need = topk_groups_ws_bytes(M, N);
    if (!ws || !aligned(ws, 16) || ws_bytes < need)
        return fail(DB_ENOSPC, "emb_topk_groups: workspace %zu bytes < %zu needed (16-byte "
                    "aligned)", ws ? ws_bytes : 0, need);
    hipError_t e = launch_topk_groups(M, N, k, D, ws, idx, d, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_topk_groups: launch");
    return DB_OK;
}

size_t emb_topk_min_workspace_bytes(int M, int N, int k)
{
    if (M <= 0 || N <= 0 || k < 1 || k > N || k > DB_KMAX) return 0;
    return topk_min_ws_bytes(M, N, k);
}

int emb_topk_min(int M, int N, const float *D, int k, int32_t *idx, float *d, void *ws,
                 size_t ws_bytes, void *stream)
{
    if (M <= 0 || N <= 0 || !D || !idx || !d || k < 1 || k > N || k > DB_KMAX)
        return fail(DB_EINVAL, "emb_topk_min: bad arguments (k = %d, N = %d)", k, N);
    if (ws && !aligned(ws, 16)) return fail(DB_EINVAL, "emb_topk_min: workspace not 16-byte aligned");
    hipError_t e = launch_topk_min(M, N, k, D, idx, d, ws, ws_bytes,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_topk_min: launch");
    return DB_OK;
}

// Rerank workspace: packed queries, per-block counts, query counts, row boxes.
size_t emb_knn_workspace_bytes(int M, int N, int k)
{
    if (M <= 0 || N <= 0 || k < 1 || k > kKnnMaxKPublic || k > N) return 0;
    return knn_ws_bytes(M, N);
}

int emb_knn(int fmt, int M, int N, int dim, const void *q_codes, const float *q_scale,
            const float *q_sq, const void *x_codes, const float *x_scale, const float *x_sq, int k,
            int direct, int32_t *idx, float *d, void *ws, size_t ws_bytes, void *stream)
{
    if (fmt == EMB_BIN) return fail(DB_EINVAL, "emb_knn: BF16 or FP8 latents only");
    int rc = dist_check("emb_knn", fmt, M, N, dim, q_codes, q_scale, q_sq, x_codes, x_scale,
                        x_sq, d);
    if (rc) return rc;
    if (k < 1 || k > kKnnMaxKPublic || k > N || !idx)
        return fail(DB_EINVAL, "emb_knn: k = %d outside [1, min(N, %d)] or idx NULL", k,
                    kKnnMaxKPublic);
    if ((int64_t)N * dim * (fmt == EMB_BF16 ? 2 : 1) >= ((int64_t)1 << 32))
        return fail(DB_EINVAL, "emb_knn: database codes must stay below 4 GiB");
    const size_t need = knn_ws_bytes(M, N);
    if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
        return fail(DB_ENOSPC, "emb_knn: workspace %zu bytes < %zu needed (256-byte aligned)",
                    ws ? ws_bytes : (size_t)0, need);
    hipError_t e = launch_knn(fmt == EMB_FP8, M, N, dim, q_codes, q_scale, q_sq, x_codes, x_scale,
                              x_sq, k, direct != 0, idx, d, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "emb_knn: launch");
    return DB_OK;
}

static size_t rerank_layout(const db_t *db, int nq, size_t *o_qpack, size_t *o_qpart,
                            size_t *o_acnt, size_t *o_box, size_t *o_mom = nullptr,
                            size_t *o_scored = nullptr, size_t *o_tbox = nullptr)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    *o_qpack = take((size_t)nq * 2 * db->g.Wp * 4);
    *o_qpart = take((size_t)nq * kQueryParts * sizeof(QueryPart));
    *o_acnt = take((size_t)nq * 2 * 4);
    *o_box = take((size_t)nq * 4 * 4);
    const size_t om = take((size_t)nq * 4 * 8);
    if (o_mom) *o_mom = om;
    const size_t osc = take(rerank_ws_bytes(nq));
    if (o_scored) *o_scored = osc;
    const size_t otb = take((size_t)nq * 4 * 4);
    if (o_tbox) *o_tbox = otb;
    return off;
}

size_t db_rerank_workspace_bytes(const db_t *db, int nq)
{
    if (!live(db) || nq <= 0) return 0;
    size_t a, b, c, d;
    return rerank_layout(db, nq, &a, &b, &c, &d);
}

// Score the candidates (the dominant kernel of a rerank: profiled), then rank them.
static hipError_t rerank_launches(const db_t *db, int nq, const uint32_t *qpack,
                                  const uint32_t *acnt, const int32_t *box, const int32_t *tbox,
                                  const int32_t *cand, int nc, int k, int32_t *idx, double *score,
                                  db_counts_t *counts, void *ws, hipStream_t s)
{
    hipError_t e = prof_mark(db, s);
    if (e == hipSuccess) e = launch_rerank_score(db, nq, qpack, acnt, box, tbox, cand, nc, k, ws, s);
    if (e == hipSuccess) e = prof_mark(db, s);
    if (e == hipSuccess) e = launch_rerank_rank(db, nq, acnt, nc, k, idx, score, counts, ws, s);
    return e;
}

// Pack the queries into the rerank workspace: bit planes, counts, row boxes, moments;
// with pooled, also the labels' pooled counts for the encoder.
static hipError_t enqueue_rerank_pack(const db_t *db, int nq, const uint8_t *q_labels, void *ws,
                                      hipStream_t s, uint8_t *pooled = nullptr)
{
    size_t oq, op, oa, ob, om, osc, otb;
    rerank_layout(db, nq, &oq, &op, &oa, &ob, &om, &osc, &otb);
    hipError_t e = pooled ? launch_pack_pool_queries(db, q_labels, nq, at<uint32_t>(ws, oq),
                                                     at<QueryPart>(ws, op), pooled, s)
                          : launch_pack_queries(db, q_labels, nq, nullptr, at<uint32_t>(ws, oq),
                                                at<QueryPart>(ws, op), s);
    if (e == hipSuccess)
        e = launch_sum_parts(at<QueryPart>(ws, op), nq, at<uint32_t>(ws, oa), at<int32_t>(ws, ob),
                             at<uint64_t>(ws, om), s, at<int32_t>(ws, otb));
    return e;
}

// Score and rank the candidates of queries packed into ws.
static hipError_t enqueue_rerank_score(const db_t *db, int nq, const int32_t *cand, int nc, int k,
                                       int32_t *idx, double *score, db_counts_t *counts, void *ws,
                                       hipStream_t s)
{
    size_t oq, op, oa, ob, om, osc, otb;
    rerank_layout(db, nq, &oq, &op, &oa, &ob, &om, &osc, &otb);
    return rerank_launches(db, nq, at<uint32_t>(ws, oq), at<uint32_t>(ws, oa), at<int32_t>(ws, ob),
                           at<int32_t>(ws, otb), cand, nc, k, idx, score, counts,
                           at<char>(ws, osc), s);
}

static hipError_t enqueue_rerank(const db_t *db, int nq, const uint8_t *q_labels,
                                 const int32_t *cand, int nc, int k, int32_t *idx, double *score,
                                 db_counts_t *counts, void *ws, hipStream_t s)
{
    hipError_t e = enqueue_rerank_pack(db, nq, q_labels, ws, s);
    if (e == hipSuccess) e = enqueue_rerank_score(db, nq, cand, nc, k, idx, score, counts, ws, s);
    return e;
}

int db_rerank_pack(const db_t *db, int nq, const uint8_t *q_labels, void *ws, size_t ws_bytes,
                   void *stream)
{
    int rc = check_query_common("db_rerank_pack", db, q_labels, ws);
    if (rc) return rc;
    if (nq <= 0) return fail(DB_EINVAL, "db_rerank_pack: nq %d", nq);
    const size_t need = db_rerank_workspace_bytes(db, nq);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_rerank_pack: workspace %zu bytes < %zu needed", ws_bytes, need);
    hipError_t e = enqueue_rerank_pack(db, nq, q_labels, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "db_rerank_pack: launch");
    return DB_OK;
}

int db_rerank_pack_pool(const db_t *db, int nq, const uint8_t *q_labels, uint8_t *pooled,
                        void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_rerank_pack_pool", db, q_labels, ws);
    if (rc) return rc;
    if (nq <= 0) return fail(DB_EINVAL, "db_rerank_pack_pool: nq %d", nq);
    if (db->g.ny % 2 || db->g.nz % 2)
        return fail(DB_EINVAL, "db_rerank_pack_pool: grid %d x %d x %d: ny and nz must be even",
                    db->g.nx, db->g.ny, db->g.nz);
    if (!pooled || !aligned(pooled, 8))
        return fail(DB_EINVAL, "db_rerank_pack_pool: pooled must be non-NULL and 8-byte aligned");
    const size_t need = db_rerank_workspace_bytes(db, nq);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_rerank_pack_pool: workspace %zu bytes < %zu needed", ws_bytes,
                    need);
    hipError_t e = enqueue_rerank_pack(db, nq, q_labels, ws, static_cast<hipStream_t>(stream),
                                       pooled);
    if (e != hipSuccess) return hip_fail(e, "db_rerank_pack_pool: launch");
    return DB_OK;
}

int db_rerank_packed(const db_t *db, int nq, const int32_t *cand, int nc, int k, int32_t *idx,
                     double *score, db_counts_t *counts, void *ws, size_t ws_bytes, void *stream)
{
    if (!live(db)) return fail(DB_ESTATE, "db_rerank_packed: invalid handle");
    if (db->count <= 0) return fail(DB_EINVAL, "db_rerank_packed: database is empty");
    if (!ws || !aligned(ws, kAlign))
        return fail(DB_EINVAL, "db_rerank_packed: workspace must be non-NULL and 256-byte aligned");
    if (nq <= 0 || !cand || !idx || !score || nc < 1 || nc > DB_KMAX || k < 1 || k > nc)
        return fail(DB_EINVAL, "db_rerank_packed: bad arguments (nq %d, nc %d, k %d)", nq, nc, k);
    const size_t need = db_rerank_workspace_bytes(db, nq);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_rerank_packed: workspace %zu bytes < %zu needed", ws_bytes, need);
    hipError_t e = enqueue_rerank_score(db, nq, cand, nc, k, idx, score, counts, ws,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "db_rerank_packed: launch");
    return DB_OK;
}

int db_rerank(const db_t *db, int nq, const uint8_t *q_labels, const int32_t *cand, int nc, int k,
              int32_t *idx, double *score, db_counts_t *counts, void *ws, size_t ws_bytes,
              void *stream)
{
    int rc = check_query_common("db_rerank", db, q_labels, ws);
    if (rc) return rc;
    if (nq <= 0 || !cand || !idx || !score || nc < 1 || nc > DB_KMAX || k < 1 || k > nc)
        return fail(DB_EINVAL, "db_rerank: bad arguments (nq %d, nc %d, k %d)", nq, nc, k);
    const size_t need = db_rerank_workspace_bytes(db, nq);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_rerank: workspace %zu bytes < %zu needed", ws_bytes, need);
    hipError_t e = enqueue_rerank(db, nq, q_labels, cand, nc, k, idx, score, counts, ws,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "db_rerank: launch");
    return DB_OK;
}

// Workspace of db_query_embed: one region used either by the fused nearest-latent search
// (its lists) or by the distance matrix and its selection workspace (binary codes, or
// n_cand above the fused search's limit), then the candidates and the rerank's part.
static size_t embed_layout(const db_t *db, int nq, int n_cand, size_t *o_D, size_t *o_ci,
                           size_t *o_cd, size_t *o_rr, size_t *o_sel = nullptr,
                           size_t *sel_bytes = nullptr)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    const int ncap = db->capacity > INT32_MAX ? INT32_MAX : (int)db->capacity;
    const size_t dbytes = align_up((size_t)nq * db->capacity * 4, kAlign);
    const size_t sb = n_cand <= ncap ? std::max(topk_min_ws_bytes(nq, ncap, n_cand),
                                                topk_groups_ws_bytes(nq, ncap))
                                     : 0;
    const size_t kb = n_cand <= kKnnMaxKPublic ? knn_ws_bytes(nq, ncap) : 0;
    *o_D = take(std::max(dbytes + sb, kb));
    *o_ci = take((size_t)nq * n_cand * 4);
    *o_cd = take((size_t)nq * n_cand * 4);
    size_t a, b, c, d;
    *o_rr = take(rerank_layout(db, nq, &a, &b, &c, &d));
    if (o_sel) *o_sel = *o_D + dbytes;
    if (sel_bytes) *sel_bytes = sb;
    return off;
}

size_t db_query_embed_workspace_bytes(const db_t *db, int nq, int n_cand)
{
    if (!live(db) || nq <= 0 || n_cand <= 0) return 0;
    size_t a, b, c, d;
    return embed_layout(db, nq, n_cand, &a, &b, &c, &d);
}

int db_query_embed(const db_t *db, int fmt, int nq, int dim, const void *q_codes,
                   const float *q_scale, const float *q_sq, const void *x_codes,
                   const float *x_scale, const float *x_sq, const uint8_t *q_labels, int n_cand,
                   int k, int32_t *idx, double *score, db_counts_t *counts, int32_t *cand_idx,
                   float *cand_d, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_query_embed", db, q_labels, ws);
    if (rc) return rc;
    const int64_t n = db->count;
    if (nq <= 0 || n_cand < 1 || n_cand > DB_KMAX || n_cand > n || k < 1 || k > n_cand || !idx ||
        !score || n > INT32_MAX)
        return fail(DB_EINVAL, "db_query_embed: bad arguments (nq %d, n_cand %d, k %d)", nq,
                    n_cand, k);
    size_t oD, oci, ocd, orr;
    const size_t need = embed_layout(db, nq, n_cand, &oD, &oci, &ocd, &orr);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_query_embed: workspace %zu bytes < %zu needed", ws_bytes, need);
    float *D = at<float>(ws, oD);
    int32_t *ci = cand_idx ? cand_idx : at<int32_t>(ws, oci);
    float *cd = cand_d ? cand_d : at<float>(ws, ocd);
    size_t osel, sel_bytes;
    embed_layout(db, nq, n_cand, &oD, &oci, &ocd, &orr, &osel, &sel_bytes);
    void *sel = sel_bytes ? at<char>(ws, osel) : nullptr;
    if (fmt != EMB_BIN && n_cand <= kKnnMaxKPublic) {
        // Distances and the nearest n_cand in one pass (no distance matrix); the reported
        // candidate distances are recomputed in direct form.
        rc = emb_knn(fmt, nq, (int)n, dim, q_codes, q_scale, q_sq, x_codes, x_scale, x_sq,
                     n_cand, 1, ci, cd, at<char>(ws, oD), knn_ws_bytes(nq, (int)n), stream);
    } else if (fmt != EMB_BIN && sel && sel_bytes >= topk_groups_ws_bytes(nq, (int)n)) {
        // Distances with their group minima, then the bound read from those.
        rc = emb_distances_groups(fmt, nq, (int)n, dim, q_codes, q_scale, q_sq, x_codes, x_scale,
                                  x_sq, D, sel, sel_bytes, stream);
        if (rc) return rc;
        rc = emb_topk_groups(nq, (int)n, D, n_cand, ci, cd, sel, sel_bytes, stream);
    } else {
        rc = emb_distances(fmt, nq, (int)n, dim, q_codes, q_scale, q_sq, x_codes, x_scale, x_sq,
                           D, stream);
        if (rc) return rc;
        rc = emb_topk_min(nq, (int)n, D, n_cand, ci, cd, sel, sel_bytes, stream);
    }
    if (rc) return rc;
    hipError_t e = enqueue_rerank(db, nq, q_labels, ci, n_cand, k, idx, score, counts,
                                  at<char>(ws, orr), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "db_query_embed: rerank launch");
    return DB_OK;
}

// ---- centre-of-mass prefilter + exact rerank ----

static size_t com_layout(const db_t *db, int nq, int n_cand, size_t *o_D, size_t *o_ci,
                         size_t *o_cd, size_t *o_rr)
{
    return embed_layout(db, nq, n_cand, o_D, o_ci, o_cd, o_rr);
}

size_t db_query_com_workspace_bytes(const db_t *db, int nq, int n_cand)
{
    if (!live(db) || nq <= 0 || n_cand <= 0) return 0;
    size_t a, b, c, d;
    return com_layout(db, nq, n_cand, &a, &b, &c, &d);
}

int db_query_com(const db_t *db, int nq, const uint8_t *q_labels, int n_cand, int k, int32_t *idx,
                 double *score, db_counts_t *counts, int32_t *cand_idx, float *cand_d, void *ws,
                 size_t ws_bytes, void *stream)
{
    int rc = check_query_common("db_query_com", db, q_labels, ws);
    if (rc) return rc;
    const int64_t n = db->count;
    if (nq <= 0 || nq > 65535 || n_cand < 1 || n_cand > DB_KMAX || n_cand > n || k < 1 ||
        k > n_cand || !idx || !score || n > INT32_MAX)
        return fail(DB_EINVAL, "db_query_com: bad arguments (nq %d, n_cand %d, k %d)", nq,
                    n_cand, k);
    size_t oD, oci, ocd, orr;
    const size_t need = com_layout(db, nq, n_cand, &oD, &oci, &ocd, &orr);
    if (ws_bytes < need)
        return fail(DB_ENOSPC, "db_query_com: workspace %zu bytes < %zu needed", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *D = at<float>(ws, oD);
    int32_t *ci = cand_idx ? cand_idx : at<int32_t>(ws, oci);
    float *cd = cand_d ? cand_d : at<float>(ws, ocd);
    char *rr = at<char>(ws, orr);
    size_t oq, op, oa, ob, om, osc, otb;
    rerank_layout(db, nq, &oq, &op, &oa, &ob, &om, &osc, &otb);
    uint32_t *qpack = at<uint32_t>(rr, oq);
    uint32_t *acnt = at<uint32_t>(rr, oa);
    int32_t *box = at<int32_t>(rr, ob), *tbox = at<int32_t>(rr, otb);
    uint64_t *qmom = at<uint64_t>(rr, om);
    QueryPart *qpart = at<QueryPart>(rr, op);
    hipError_t e = launch_pack_queries(db, q_labels, nq, nullptr, qpack, qpart, s);
    if (e == hipSuccess) e = launch_sum_parts(qpart, nq, acnt, box, qmom, s, tbox);
    if (e == hipSuccess) e = launch_com_dist(nq, qmom, db->mom, (int)n, D, s);
    size_t osel, sel_bytes;
    embed_layout(db, nq, n_cand, &oD, &oci, &ocd, &orr, &osel, &sel_bytes);
    if (e == hipSuccess)
        e = launch_topk_min(nq, (int)n, n_cand, D, ci, cd, sel_bytes ? at<char>(ws, osel) : nullptr,
                            sel_bytes, s);
    if (e == hipSuccess)
        e = rerank_launches(db, nq, qpack, acnt, box, tbox, ci, n_cand, k, idx, score, counts,
                            at<char>(rr, osc), s);
    if (e != hipSuccess) return hip_fail(e, "db_query_com: launch");
    return DB_OK;
}

// ---- order-0 resampling ----

// Output voxel o of an axis of n_out samples reads source voxel
// round(o * (n_in - 1) / (n_out - 1)), in exact integer arithmetic.
static bool fill_map(uint16_t *map, int n_in, int n_out)
{
    if (n_out < 1 || n_out > kMaxResample || n_in < 1 || n_in > 65535) return false;
    for (int o = 0; o < n_out; ++o) {
        const int64_t num = 2 * (int64_t)o * (n_in - 1) + (n_out - 1);
        map[o] = (uint16_t)(n_out == 1 ? 0 : num / (2 * (int64_t)(n_out - 1)));
    }
    return true;
}

int db_append_resampled(db_t *dst, const db_t *src, int64_t first, int64_t n, void *stream)
{
    if (!live(dst) || !live(src)) return fail(DB_ESTATE, "db_append_resampled: invalid handle");
    if (first < 0 || n < 0 || first + n > src->count)
        return fail(DB_EINVAL, "db_append_resampled: entries [%lld, %lld) outside the source",
                    (long long)first, (long long)(first + n));
    if (n == 0) return DB_OK;
    if (dst->count + n > dst->capacity)
        return fail(DB_ENOSPC, "db_append_resampled: capacity %lld exceeded",
                    (long long)dst->capacity);
    if (dst->t_lo != src->t_lo || dst->t_hi != src->t_hi)
        return fail(DB_EINVAL, "db_append_resampled: thresholds of the two databases differ");
    ResampleMaps maps;
    if (!fill_map(maps.x, src->g.nx, dst->g.nx) || !fill_map(maps.y, src->g.ny, dst->g.ny) ||
        !fill_map(maps.z, src->g.nz, dst->g.nz))
        return fail(DB_EINVAL, "db_append_resampled: output axes must be 1..%d voxels",
                    kMaxResample);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_resample_db(src, first, n, dst, maps, s);
    if (e == hipSuccess)
        e = launch_meta(dst->planes + dst->count * 2 * (int64_t)dst->g.Wp, n, dst->g,
                        dst->box + dst->count * 4, dst->tbox + dst->count * 4,
                        dst->mom + dst->count * 4, dst->zrange + dst->count * dst->g.nz * 2, s);
    if (e == hipSuccess)
        e = launch_block_counts(dst, dst->planes + dst->count * 2 * (int64_t)dst->g.Wp, n,
                                dst->box + dst->count * 4, block_counts_at(dst, dst->count), s);
    if (e != hipSuccess) return hip_fail(e, "db_append_resampled: launch");
    dst->count += n;
    return DB_OK;
}

int labels_resample(int nq, const uint8_t *in, int nx, int ny, int nz, uint8_t *out, int mx,
                    int my, int mz, void *stream)
{
    if (nq <= 0 || !in || !out || nx <= 0 || ny <= 0 || nz <= 0)
        return fail(DB_EINVAL, "labels_resample: bad arguments");
    ResampleMaps maps;
    if (!fill_map(maps.x, nx, mx) || !fill_map(maps.y, ny, my) || !fill_map(maps.z, nz, mz))
        return fail(DB_EINVAL, "labels_resample: output axes must be 1..%d voxels", kMaxResample);
    hipError_t e = launch_resample_labels(nq, in, nx, ny, nz, out, mx, my, mz, maps,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "labels_resample: launch");
    return DB_OK;
}

int db_sync(const db_t *db, void *stream)
{
    if (!live(db)) return fail(DB_ESTATE, "db_sync: invalid handle");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "db_sync");
    return DB_OK;
}

int db_set_rerank_bound(db_t *db, int on)
{
    if (!live(db)) return fail(DB_EINVAL, "db_set_rerank_bound: invalid handle");
    db->rerank_bound = on ? 1 : 0;
    return DB_OK;
}

int db_tune_batch(db_t *db, int slab_planes, int block_threads, int tile_entries,
                  int query_chunk)
{
    if (!live(db)) return fail(DB_ESTATE, "db_tune_batch: invalid handle");
    if (slab_planes < -1 || slab_planes > db->g.nz)
        return fail(DB_EINVAL, "db_tune_batch: slab_planes %d outside [-1, %d]", slab_planes,
                    db->g.nz);
    if (block_threads != 0 && block_threads != 256 && block_threads != 512 &&
        block_threads != 1024)
        return fail(DB_EINVAL, "db_tune_batch: block_threads must be 0, 256, 512 or 1024");
    if (tile_entries != 0 && tile_entries != 4 && tile_entries != 8)
        return fail(DB_EINVAL, "db_tune_batch: tile_entries must be 0, 4 or 8");
    if (query_chunk < 0 || query_chunk > 1024)
        return fail(DB_EINVAL, "db_tune_batch: query_chunk %d outside [0, 1024]", query_chunk);
    db->batch_planes = slab_planes;
    db->batch_threads = block_threads;
    db->batch_tile = tile_entries;
    db->batch_qchunk = query_chunk;
    return DB_OK;
}

int db_profile(db_t *db, int enable)
{
    if (!live(db)) return fail(DB_ESTATE, "db_profile: invalid handle");
    if (!db->prof) {
        db->prof = new (std::nothrow) Profiler();
        if (!db->prof) return fail(DB_ENOMEM, "db_profile: out of host memory");
    }
    db->prof->on = enable != 0;
    return DB_OK;
}

int db_profile_read(db_t *db, double *ms, int64_t *launches)
{
    if (!live(db)) return fail(DB_ESTATE, "db_profile_read: invalid handle");
    if (!ms || !launches) return fail(DB_EINVAL, "db_profile_read: NULL output");
    double total = 0.0;
    int64_t n = 0;
    if (db->prof) {
        Profiler &P = *db->prof;
        for (size_t i = 0; i + 1 < P.used; i += 2) {
            hipError_t e = hipEventSynchronize(P.ev[i + 1]);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, P.ev[i], P.ev[i + 1]);
            if (e != hipSuccess) return hip_fail(e, "db_profile_read");
            total += t;
            ++n;
        }
        P.used = 0;
    }
    *ms = total;
    *launches = n;
    return DB_OK;
}

void db_free(db_t *db)
{
    if (!live(db)) return;
    delete db->graph;
    delete db->prof;
    db->magic = 0;
    delete db;
}

const char *db_last_error(void) { return g_err; }

}  // extern "C"
