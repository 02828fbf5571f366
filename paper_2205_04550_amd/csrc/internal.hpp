// internal.hpp — handle layout, workspace layout and kernel launchers of libtumordb.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tumordb.h"

namespace tdb {

constexpr uint64_t kMagic = 0x7475'6d6f'7264'6231ULL;  // "tumordb1"
constexpr size_t kAlign = 256;
constexpr int kQueryParts = 64;     // blocks of the query-pack kernel
constexpr int kTopkChunk = 2048;    // entries one top-k block ranks at a time

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Geometry {
    int nx, ny, nz;
    int64_t V;   // voxels
    int W;       // words per mask plane (V / 32)
    int Wp;      // padded to a multiple of 4 words (16 bytes)
    int nxw;     // words per x-row (nx / 32)
};

bool make_geometry(int nx, int ny, int nz, Geometry *g);

// The 16^3-voxel blocks of the per-entry counts that bound a candidate's Dice score in the
// rerank: nbx = 2 nxw x blocks, ceil(ny / 16) y blocks, ceil(nz / 16) z blocks; returns the
// blocks per mask padded to a multiple of 8, or 0 (no counts kept) above kBoundMaxBlocks.
constexpr int kBoundMaxBlocks = 2048;
inline int bound_blocks(const Geometry &g, int *nbx, int *nby)
{
    const int bx = 2 * g.nxw, by = (g.ny + 15) / 16, bz = (g.nz + 15) / 16;
    if (nbx) *nbx = bx;
    if (nby) *nby = by;
    const int64_t nb = (int64_t)bx * by * bz;
    return nb <= kBoundMaxBlocks ? (int)((nb + 7) / 8 * 8) : 0;
}

// Error reporting shared by every C entry point (message read by db_last_error).
int tdb_set_error(int code, const char *fmt, ...);
bool tdb_live(const db_t *db);

struct BatchGraph;  // cached HIP graph of a batched query (api.cpp)
struct Profiler;    // HIP events around the dominant kernel (api.cpp)

}  // namespace tdb

struct db_t {
    uint64_t magic;
    tdb::Geometry g;
    float t_lo, t_hi;
    int64_t capacity, count;
    uint32_t *planes;   // [capacity][2][Wp]
    uint32_t *popcnt;   // [capacity][2]
    int32_t *box;       // [capacity][4] row box z0, z1, y0, y1 of the set bits
    int32_t *tbox;      // [capacity][4] row box of the T1Gd bits alone (all zero: none)
    uint32_t *zrange;   // [capacity][nz][2] per z-slice y-range of the FLAIR / T1Gd rows
    uint16_t *bcnt;     // [capacity][2][nbp] set voxels per 16^3 block (nbp = bound_blocks)
    int rerank_bound;   // 1: the rerank scores candidates in bound order and skips the rest
    uint64_t *mom;      // [capacity][4] FLAIR moments: sum x, sum y, sum z, count
    int32_t *tile_order;  // [capacity] entries sorted by row-box centre, in tiles by cost
    int64_t tile_order_n; // entries the tile order covers (it is rebuilt when count differs)
    int tile_order_tile;  // entries per tile it was built for
    size_t storage_bytes;
    int cus;                 // compute units of the device the handle was built on
    int device;
    int lds_max;             // LDS bytes one block may use on that device
    int batch_planes;        // tuned z-planes per LDS slab of the batched scan (0 = most that fit)
    int batch_threads;       // tuned block size of the batched scan (0 = default)
    int batch_tile;          // tuned entries per tile (0 = 4; 4 or 8)
    int batch_qchunk;        // tuned queries per chunk (0 = 256)
    tdb::BatchGraph *graph;
    tdb::Profiler *prof;
};

namespace tdb {

// Offsets of the pieces of a query workspace (bytes from its base).
struct WsLayout {
    size_t qpack;    // uint32 [nq][2][Wp] packed (and ROI-masked) queries
    size_t qpart;    // QueryPart [nq][kQueryParts] per-block query partials
    size_t acnt;     // uint32 [nq][2] query counts |A_m (n R)|
    size_t rois;     // int32 [nq][6] ROI boxes (batched calls)
    size_t qbox;     // int32 [nq][4] row boxes of the packed queries
    size_t qtbox;    // int32 [nq][4] row boxes of their T1Gd bits alone
    size_t qmom;     // uint64 [nq][4] FLAIR moments of the packed queries
    size_t inter;    // uint32 [nq][capacity][2] intersections
    size_t bcnt;     // uint32 [nq][capacity][2] database counts inside the ROI (batched)
    size_t plan;     // int32: query order [nq], queue counters [8], slab lists (batched)
    size_t topk_a;   // ping-pong top-k candidate buffers: uint64 score bits + int32 index
    size_t topk_b;
    size_t total;
};

// What one block of the query-pack kernel found in its share of a query's words.
struct QueryPart {
    uint32_t cnt[2];   // set bits of the FLAIR and T1Gd masks
    int32_t box[4];    // z min, z max, y min, y max of rows with a set bit (INT_MAX/-1: none)
    int32_t tbox[4];   // the same for the rows with a T1Gd bit
    uint64_t mom[3];   // sum of x, y, z over the FLAIR bits
};

WsLayout ws_layout(const db_t *db, int nq, int k, bool batched);
// One exact query (pack, scan, Dice + top-k) enqueued on s into ws laid out as L
// (ws_layout(db, 1, k, .)); arguments checked by check_query_args beforehand.
hipError_t enqueue_query(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx,
                         double *score, db_counts_t *counts, void *ws, const WsLayout &L,
                         hipStream_t s);
int check_query_args(const char *fn, const db_t *db, const uint8_t *q_labels, int k,
                     const int32_t *idx, const double *score);
int64_t topk_blocks(int64_t n);

// ---- launchers (each returns hipGetLastError of its launch) ----
hipError_t launch_pack_db(const db_t *db, const float *conc, int64_t n, uint32_t *planes,
                          uint32_t *popcnt, hipStream_t s);
hipError_t launch_pack_queries(const db_t *db, const uint8_t *labels, int nq, const int32_t *rois,
                               uint32_t *qpack, QueryPart *qpart, hipStream_t s);
// launch_pack_queries without ROI that also writes the labels' 2x2x2 pooled counts,
// uint8 [nq][nz/2][ny/2][nx/2] (FLAIR count bits 0..3, T1Gd count bits 4..7); ny, nz even.
hipError_t launch_pack_pool_queries(const db_t *db, const uint8_t *labels, int nq,
                                    uint32_t *qpack, QueryPart *qpart, uint8_t *pooled,
                                    hipStream_t s);
// Per query: counts acnt [nq][2], row box qbox [nq][4] (z0, z1, y0, y1; all zero when
// empty), FLAIR moments qmom [nq][4] (sum x, sum y, sum z, count) and, unless qtbox is NULL,
// the row box of the T1Gd bits alone qtbox [nq][4].
hipError_t launch_sum_parts(const QueryPart *qpart, int nq, uint32_t *acnt, int32_t *qbox,
                            uint64_t *qmom, hipStream_t s, int32_t *qtbox = nullptr);
hipError_t launch_scan(const db_t *db, int64_t n, const uint32_t *qpack, uint32_t *inter,
                       hipStream_t s);
// Shape of a batched launch: LDS slabs of Z planes (use_lds) or the L2 fallback.
struct BatchPlan {
    bool use_lds;
    int Z, nslabs, qchunk, nchunks, threads, tile;
    size_t lds_bytes;
};
BatchPlan batch_plan(const db_t *db, int nq);
int batch_tile(const db_t *db);   // entries per tile of the LDS kernel (4 or 8)
hipError_t batch_set_lds_limit(int bytes);
hipError_t launch_batch_scan(const db_t *db, int64_t n, int nq, const BatchPlan &p,
                             const uint32_t *qpack, const int32_t *rois, const int32_t *order,
                             const int32_t *list_off, const int32_t *list_q, int32_t *counters,
                             uint32_t *inter, uint32_t *bcnt, hipStream_t s);
hipError_t launch_fill_u32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Embedding search (embed.hip).
hipError_t launch_quant_bf16(int64_t n, int dim, const float *x, uint16_t *y, float *sq,
                             hipStream_t s);
hipError_t launch_quant_fp8(int64_t n, int dim, const float *x, uint8_t *y, float *scale,
                            float *sq, hipStream_t s);
// mode 0: squared L2; 1: L2; 2: add L2 to D. gmin (mode 0 only, else NULL): also the
// minimum key of every whole group of 16 entries of each row, [M][N / 16], for
// launch_topk_groups.
hipError_t launch_dist_bf16(int M, int N, int K, const uint16_t *Q, const float *qn,
                            const uint16_t *X, const float *xn, float *D, int mode,
                            uint32_t *gmin, hipStream_t s);
hipError_t launch_dist_fp8(int M, int N, int K, const uint8_t *Q, const float *qs, const float *qn,
                           const uint8_t *X, const float *xs, const float *xn, float *D,
                           int mode, uint32_t *gmin, hipStream_t s);
// k smallest per row of D [M][N] from the group minima a distance launch left in ws
// (topk_groups_ws_bytes; the minima at topk_groups_gmin(ws, M)); one block per row
// when no bound applies to (N, k).
size_t topk_groups_ws_bytes(int M, int N);
uint32_t *topk_groups_gmin(void *ws, int M);
hipError_t launch_topk_groups(int M, int N, int k, const float *D, void *ws, int32_t *idx,
                              float *d, hipStream_t s);
// k smallest per row of D [M][N]. With a workspace of topk_min_ws_bytes (> 0) the rows
// are split into chunks selected in parallel and merged; without, one block per row.
size_t topk_min_ws_bytes(int M, int N, int k);
hipError_t launch_topk_min(int M, int N, int k, const float *D, int32_t *idx, float *d, void *ws,
                           size_t ws_bytes, hipStream_t s);
// Fused distances + k nearest per query (knn.hip): k <= knn_max_k(), no distance matrix.
// ws of knn_ws_bytes(M, N) bytes (256-byte aligned). direct: d holds the direct-form
// distances of the selected pairs (float64 sum, rounded once) instead of the expanded ones.
constexpr int kKnnMaxKPublic = 256;
size_t knn_ws_bytes(int M, int N);
hipError_t launch_knn(bool fp8, int M, int N, int K, const void *Q, const float *qs,
                      const float *qn, const void *X, const float *xs, const float *xn, int k,
                      bool direct, int32_t *idx, float *d, void *ws, hipStream_t s);
// Exact rerank of nc <= DB_KMAX candidates per query; ws of rerank_ws_bytes(nq) holds the
// scored candidates between the scoring and the ranking kernel.
size_t rerank_ws_bytes(int nq);
// box: the queries' row boxes; tbox: those of their T1Gd bits alone (the T1Gd plane of a
// pair is read only inside both T1Gd boxes).
// With the block counts kept and k <= 64, the candidates go in bound order: the first
// max(16, k) rounded to 16 are scored, then those whose bound reaches the k-th best score.
hipError_t launch_rerank_score(const db_t *db, int nq, const uint32_t *qpack, const uint32_t *acnt,
                               const int32_t *box, const int32_t *tbox, const int32_t *cand,
                               int nc, int k, void *ws, hipStream_t s);
// The 16^3-block counts of n entries (planes, row boxes) into bcnt.
hipError_t launch_block_counts(const db_t *db, const uint32_t *planes, int64_t n,
                               const int32_t *box, uint16_t *bcnt, hipStream_t s);
hipError_t launch_rerank_rank(const db_t *db, int nq, const uint32_t *acnt, int nc, int k,
                              int32_t *idx, double *score, db_counts_t *counts, const void *ws,
                              hipStream_t s);

// Row boxes, moments, box-restricted scan, centre-of-mass distances (sparse.hip).
// Per entry of recs: box (rows with a set bit), tbox (rows with a T1Gd bit), mom, and the
// per z-slice y-ranges of its FLAIR and T1Gd rows zrange [nz][2] (y0 | y1 << 16; 0: none).
hipError_t launch_meta(const uint32_t *recs, int64_t n, const Geometry &g, int32_t *box,
                       int32_t *tbox, uint64_t *mom, uint32_t *zrange, hipStream_t s);
// qtbox: the query's T1Gd row box (the T1Gd plane is read only inside both T1Gd boxes).
hipError_t launch_box_scan(const db_t *db, int64_t n, const uint32_t *qpack, const int32_t *qbox,
                           const int32_t *qtbox, uint32_t *inter, hipStream_t s);
hipError_t launch_com_dist(int nq, const uint64_t *qmom, const uint64_t *mom, int n, float *D,
                           hipStream_t s);

// Binary codes, Hamming distances, Bi-half layer (hash.hip).
hipError_t launch_col_kth(const float *X, int64_t n, int dim, int64_t k, float *thr, hipStream_t s);
hipError_t launch_binarize(const float *X, int64_t n, int dim, const float *thr, uint32_t *codes,
                           hipStream_t s);
hipError_t launch_hamming(int M, int N, int words, const uint32_t *Q, const uint32_t *X, float *D,
                          hipStream_t s);
hipError_t launch_bihalf_fwd(bool f64, int B, int D, const void *U, void *out, hipStream_t s);
hipError_t launch_bihalf_bwd(bool f64, int B, int D, double gamma, const void *U, const void *Bc,
                             const void *G, void *dU, hipStream_t s);

// Order-0 resampling (resample.hip): source index of every output voxel per axis.
constexpr int kMaxResample = 256;
struct ResampleMaps {
    uint16_t x[kMaxResample], y[kMaxResample], z[kMaxResample];
};
hipError_t launch_resample_db(const db_t *src, int64_t first, int64_t n, db_t *dst,
                              const ResampleMaps &maps, hipStream_t s);
hipError_t launch_resample_labels(int nq, const uint8_t *in, int nx, int ny, int nz, uint8_t *out,
                                  int mx, int my, int mz, const ResampleMaps &maps, hipStream_t s);

// Top-k over n entries per query. inter: [nq][n..][2] with row stride
// inter_qstride; bcnt likewise (stride 0 = the database popcounts, shared).
struct TopkArgs {
    int64_t n;
    int nq, k;
    const uint32_t *inter;
    int64_t inter_qstride;   // uint32 elements between queries
    const uint32_t *bcnt;
    int64_t bcnt_qstride;
    const uint32_t *acnt;    // [nq][2]
    uint64_t *buf_s[2];
    int32_t *buf_i[2];
    int32_t *out_idx;        // [nq][k]
    double *out_score;       // [nq][k]
    db_counts_t *out_counts; // [nq][k] or null
};
hipError_t launch_topk(const TopkArgs &a, hipStream_t s);

}  // namespace tdb
