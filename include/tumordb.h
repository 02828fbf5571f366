/*
 * tumordb.h — C ABI of the MI355X tumour-database retrieval library.
 *
 * The retrieval method of "A for-loop is all you need" (arXiv 2205.04550):
 * a patient's two binary segmentations in atlas space (FLAIR and T1Gd,
 * Sec. 2.2 step 2-3 and Sec. 2.3) are compared with every pre-simulated
 * tumour of a database (Sec. 2.2 step 3). Each simulation, a density in
 * [0, 1], is thresholded into a FLAIR mask (lower threshold) and a T1Gd mask
 * (higher threshold) (Sec. 2.3); similarity is Dice_T1Gd + Dice_FLAIR and the
 * highest sum is the best match (Sec. 2.3); the exhaustive loop over the
 * database is the ground truth (Sec. 2.3, "Baseline for-loop search").
 *
 * Conventions for every call:
 *  - Grid: nx * ny * nz voxels, x fastest ([nz][ny][nx]); nx % 32 == 0.
 *  - Mask m = 0 is FLAIR (voxel c >= t_lo), m = 1 is T1Gd (c >= t_hi).
 *  - Query labels are uint8 per voxel: bit 0 FLAIR, bit 1 T1Gd; other bits
 *    are ignored.
 *  - Dice_m = 2 I_m / (A_m + B_m) in IEEE double, and 1 when A_m + B_m == 0;
 *    score = Dice_T1Gd + Dice_FLAIR (double). I, A, B are exact uint32 counts.
 *  - Ranking is a total order: score descending, then database index
 *    ascending. Indices are 0-based in insertion order.
 *  - "device" pointers are HIP device memory of the current device; the
 *    caller owns every buffer (storage, inputs, outputs, workspace). The
 *    library never allocates device memory.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream). Calls
 *    enqueue asynchronously; results are valid once the stream is synced.
 *  - Every call validates all arguments before enqueuing anything; on error
 *    it writes nothing, returns a negative code and db_last_error() explains.
 *    No C++ exception crosses this ABI. Faults of enqueued work surface at
 *    db_sync() (or the caller's own synchronisation) as DB_EHIP.
 *  - A handle is not thread-safe while db_append runs; queries on one handle
 *    may run concurrently only with distinct workspaces.
 */
#ifndef TUMORDB_H
#define TUMORDB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct db_t db_t; /* opaque handle over caller-owned device storage */

/* Half-open voxel box [x0, x1) x [y0, y1) x [z0, z1). */
typedef struct {
    int32_t x0, y0, z0, x1, y1, z1;
} db_roi_t;

/* Counts behind one score; index [0] = FLAIR, [1] = T1Gd.
 * inter = |A n B (n R)|, a = |A (n R)| (query), b = |B (n R)| (database). */
typedef struct {
    uint32_t inter[2], a[2], b[2];
} db_counts_t;

enum {
    DB_OK = 0,
    DB_EINVAL = -1, /* bad argument (null pointer, bad size, k out of range, bad ROI) */
    DB_ENOMEM = -2, /* host-side allocation failed */
    DB_EHIP = -3,   /* a HIP runtime call failed; db_last_error has its string */
    DB_ESTATE = -4, /* handle is not a live handle of this library */
    DB_ENOSPC = -5  /* storage capacity or workspace too small */
};

#define DB_KMAX 1024 /* largest k a query may request */

/* ---------------------------------------------------------------- build --- */

/* Bytes of device storage for `capacity` entries of an nx*ny*nz grid.
 * Layout (offsets from the storage base, all 256-byte aligned):
 *   planes: uint32 [capacity][2][Wp], Wp = round_up(nx*ny*nz/32, 4); word w of
 *           mask m holds voxels 32w..32w+31 of that mask, LSB first; words
 *           past nx*ny*nz/32 are zero;
 *   popcount: uint32 [capacity][2] = |B_FLAIR|, |B_T1Gd| per entry;
 *   box:      int32 [capacity][4] = z0, z1, y0, y1: the x-rows (z, y) holding
 *             any set bit of either mask lie in [z0, z1) x [y0, y1) (all zero
 *             for an entry without set bits);
 *   moments:  uint64 [capacity][4] = sum of x, of y, of z over the FLAIR
 *             voxels, and their count (the centre of mass is sum / count);
 *   order:    int32 [capacity], the entries grouped by row-box centre for
 *             db_query_batch (library-internal);
 *   tbox:     int32 [capacity][4], the box of the x-rows holding a T1Gd bit
 *             (as box, for that mask alone; the rerank reads an entry's T1Gd
 *             plane only inside it);
 *   zrange:   uint32 [capacity][nz][2]: for slice z of an entry, element 0
 *             covers the x-rows holding a FLAIR bit and element 1 those
 *             holding a T1Gd bit, as y0 | y1 << 16 with the rows in
 *             [y0, y1) (0 for a slice without such a row). The rerank and
 *             the row-box scan read a plane's row (z, y) only inside it;
 *   bcnt:     uint16 [capacity][2][nbp], the set voxels of each mask in each
 *             16 x 16 x 16 block of the grid: block (bz, by, bx) at
 *             (bz nby + by) nbx + bx with nbx = nx / 16, nby = ceil(ny / 16),
 *             nbz = ceil(nz / 16), nbp = that count rounded up to a multiple
 *             of 8 (entries past it zero); absent (0 bytes) when the grid
 *             has more than 2,048 blocks. The rerank bounds candidates by it.
 * Returns 0 if the dimensions are invalid. */
size_t db_storage_bytes(int nx, int ny, int nz, int64_t capacity);

/* Create an empty database handle over `storage` (device, >= db_storage_bytes,
 * 256-byte aligned). Thresholds t_lo < t_hi select the FLAIR and T1Gd masks
 * (Sec. 2.3: FLAIR at the lower density level, T1Gd at the higher). Nothing
 * is enqueued. The storage must outlive the handle. */
int db_build(db_t **out, int nx, int ny, int nz, float t_lo, float t_hi, int64_t capacity,
             void *storage, size_t storage_bytes);

/* Threshold and bit-pack n simulated densities (device float32 [n][nz][ny][nx],
 * 16-byte aligned) into entries db_size() .. db_size()+n-1 (Sec. 2.3: the
 * masks are extracted from the raw simulations once, before any query).
 * DB_ENOSPC if capacity would be exceeded. The input may be released once the
 * stream has passed this call. Also fills the entries' boxes and moments. */
int db_append(db_t *db, const float *conc, int64_t n, void *stream);

/* Number of entries appended so far (-1 for an invalid handle). */
int64_t db_size(const db_t *db);

/* ---------------------------------------------------------------- query --- */

/* Workspace bytes a query call needs for nq queries and top-k (0 if invalid). */
size_t db_query_workspace_bytes(const db_t *db, int nq, int k);

/* The overlap stage of one query against every entry (Sec. 2.3, baseline
 * loop): inter[n][m] = |A_m n B_m(n)| for n < db_size(), and, if qcount is
 * not NULL, qcount[m] = |A_m|. q_labels: device uint8 [nz][ny][nx];
 * inter: device uint32 [db_size()][2]; qcount: device uint32 [2] or NULL. */
int db_scan(const db_t *db, const uint8_t *q_labels, uint32_t *inter, uint32_t *qcount, void *ws,
            size_t ws_bytes, void *stream);

/* One query (Sec. 2.2 step 3 with the Sec. 2.3 score): the k best entries by
 * Dice_T1Gd + Dice_FLAIR. idx: device int32 [k]; score: device double [k];
 * counts: device db_counts_t [k] or NULL. 1 <= k <= min(db_size(), DB_KMAX). */
int db_query(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx, double *score,
             db_counts_t *counts, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory at query time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same
 * query as db_query, same arguments and results bit for bit, but without a
 * workspace argument. The workspace is carved from a fixed device array of
 * DB_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until
 * the process ends; this call allocates nothing. The database's workspace
 * (db_query_workspace_bytes without the batched parts: about 8 bytes per entry
 * of capacity plus 2 V / 8 bytes for the packed query) must fit in it, else
 * DB_ENOSPC and nothing is enqueued. The current device must be the one the
 * database was built on (DB_EINVAL otherwise). Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams, other
 * threads) race and give undefined results; calls ordered on one stream are
 * safe. The array keeps the last call's contents; each call overwrites every
 * part it reads. */
#define DB_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
int db_query_noalloc(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx, double *score,
                     db_counts_t *counts, void *stream);

/* Same contract and results, bit for bit, as db_query (same workspace size),
 * computed by reading only the x-rows where both the entry's stored box and
 * the query's box hold set bits: every other row is zero on one side and adds
 * nothing to |A_m n B_m| (Sec. 2.3, Dice). Bytes read per entry scale with
 * the tumour's extent instead of the grid (an addition to the paper's loop). */
int db_query_sparse(const db_t *db, const uint8_t *q_labels, int k, int32_t *idx, double *score,
                    db_counts_t *counts, void *ws, size_t ws_bytes, void *stream);

/* nq queries in one launch sequence, each optionally restricted to its own
 * box: both masks are cut to the box before Dice (an extension; the paper
 * compares whole volumes). The scan is one kernel launch of one block per
 * (tile of database entries, chunk of queries) item, dispatched costliest tile
 * first. q_labels: device uint8 [nq][nz][ny][nx];
 * rois: HOST array [nq] (validated before enqueue: inside the grid, non-empty)
 * or NULL for whole grids; outputs idx [nq][k], score [nq][k], counts
 * [nq][k] or NULL (device). The kernel sequence is recorded once into a HIP
 * graph per (handle, shape, pointers) and replayed. The first call after
 * entries were appended synchronises the device once to regroup the entries
 * by their row boxes. */
int db_query_batch(const db_t *db, int nq, const uint8_t *q_labels, const db_roi_t *rois, int k,
                   int32_t *idx, double *score, db_counts_t *counts, void *ws, size_t ws_bytes,
                   void *stream);

/* on = 0: the rerank (db_rerank, db_rerank_packed, db_query_embed,
 * db_query_com) scores every candidate; on != 0 (the default): in bound
 * order, leaving out those that cannot reach the top k (db_rerank). Results
 * are the same either way. DB_EINVAL on an invalid handle. */
int db_set_rerank_bound(db_t *db, int on);

/* Launch shape of db_query_batch: z-planes per LDS slab (0 = as many as fit;
 * -1 = no LDS slabs: the kernel that reads the database through L2), block
 * size (0 = 1024; else 256, 512 or 1024), database entries per tile (0 = 4;
 * 4 or 8) and queries per chunk (0 = 256; 1 .. 1024; the queries of a chunk
 * keep their counters in one block's LDS). Results do not depend on it; the
 * autotuner (paper_2205_04550_amd/autotune.py) picks it by timing. A change
 * takes effect at the next recording of the batch graph. */
int db_tune_batch(db_t *db, int slab_planes, int block_threads, int tile_entries,
                  int query_chunk);

/* ---------------------------------------------------- embedding search --- */
/* Latent search (Sec. 2.3, "Autoencoders": encoded database and query are
 * compared by L2 distance, lowest wins), then exact re-scoring of the
 * candidates with the Dice score above. Latents are row-major [n][dim]; row i
 * of the database latents belongs to entry i. Distances are the squared L2
 * distance in the expanded form |q|^2 + |x|^2 - 2 q.x, accumulated in FP32 on
 * the BF16 matrix cores: BF16 codes as stored, FP8 e4m3 codes decoded exactly
 * to BF16 (the products of codes are exact; the per-row scales multiply the
 * finished dot product). Accuracy: |d - d64| <= 1e-5 (|q|^2 + |x|^2), d64 the
 * float64 direct-form distance of the stored (dequantised) vectors. */
enum { EMB_BF16 = 0, EMB_FP8 = 1, EMB_BIN = 2 };

/* Quantise FP32 latents lat [n][dim] (device): EMB_BF16 writes uint16 codes
 * (round to nearest even); EMB_FP8 writes uint8 OCP e4m3 codes of lat/s with
 * s = max|row| / 448 (1 for a zero row) into scale[n]. sqnorm[n] = |stored
 * vector|^2 (of the dequantised values, summed in double). scale is ignored
 * for BF16. dim % 16 == 0 (BF16) or dim % 64 == 0 (FP8). */
int emb_quantize(int64_t n, int dim, const float *lat, int fmt, void *codes, float *scale,
                 float *sqnorm, void *stream);

/* D[m][n] = q_sq[m] + x_sq[n] - 2 <q_m, x_n> (FP32, device [M][N]); the
 * scales multiply the FP8 dot products and are ignored for BF16. EMB_BIN:
 * codes are dim-bit strings (uint32 [.][dim/32], see emb_binarize) and
 * D[m][n] is their Hamming distance as a float (exact); scales and squared
 * norms are ignored (may be NULL). dim % 32 == 0 and dim <= 1024 for EMB_BIN.
 * BF16 / FP8: the query codes (M x dim x 2 or 1 bytes) must stay below 2 GiB
 * (DB_EINVAL otherwise); database codes of any size are taken in chunks. */
int emb_distances(int fmt, int M, int N, int dim, const void *q_codes, const float *q_scale,
                  const float *q_sq, const void *x_codes, const float *x_scale, const float *x_sq,
                  float *D, void *stream);

/* The paper's two-encoder distance (Sec. 2.3): separate FLAIR and T1Gd
 * autoencoders give two latent sets, and a database entry's distance is the
 * sum of the two L2 distances, L2_T1Gd + L2_FLAIR (lowest wins):
 * D[m][n] = sqrt(max(d1, 0)) + sqrt(max(d2, 0)) with d1, d2 the squared
 * distances emb_distances computes for the pairs (q1, x1) and (q2, x2), in
 * that order (two launches; the second adds to D). Same fmt and dim for both
 * pairs; BF16 or FP8. */
int emb_distances_l2sum(int fmt, int M, int N, int dim, const void *q1_codes,
                        const float *q1_scale, const float *q1_sq, const void *x1_codes,
                        const float *x1_scale, const float *x1_sq, const void *q2_codes,
                        const float *q2_scale, const float *q2_sq, const void *x2_codes,
                        const float *x2_scale, const float *x2_sq, float *D, void *stream);

/* Binary codes (the paper's unsupervised hashing query, Sec. 2.3): its
 * Bi-half layer makes, per latent coordinate, the larger half of a batch +1 and
 * the rest -1, and codes are compared by L2, which for +-1 vectors is 4x their
 * Hamming distance. Here bit d of a code (LSB first in uint32 words; 1 = +1)
 * is lat[d] > thr[d], with thr[d] the lower median of coordinate d over the
 * database (the Bi-half rule with the database as the batch); queries use the
 * database's thresholds.
 * emb_hash_thresholds: thr[d] = value of 0-based rank (n - 1) / 2 in
 * ascending order of column d of lat [n][dim] (device; exact selection).
 * emb_binarize: codes [n][dim/32] (device uint32). dim % 32 == 0, dim <= 1024,
 * lat and thr 16-byte aligned. */
int emb_hash_thresholds(int64_t n, int dim, const float *lat, float *thr, void *stream);
int emb_binarize(int64_t n, int dim, const float *lat, const float *thr, uint32_t *codes,
                 void *stream);

/* Per row of D [M][N]: the k smallest values, ties by lower column, in
 * ascending order: idx [M][k] (int32), d [M][k]. 1 <= k <= min(N, DB_KMAX).
 * ws (device, 16-byte aligned) of emb_topk_min_workspace_bytes bytes lets the
 * rows be split into chunks selected by many blocks and then merged; with ws
 * NULL (or that size 0: too many candidates for the merge) one block selects
 * each row. Results are identical either way. */
size_t emb_topk_min_workspace_bytes(int M, int N, int k);
int emb_topk_min(int M, int N, const float *D, int k, int32_t *idx, float *d, void *ws,
                 size_t ws_bytes, void *stream);

/* The same distances and selection in two calls that share a workspace ws
 * (device, 16-byte aligned) of emb_groups_workspace_bytes(M, N) bytes:
 * emb_distances_groups writes D exactly as emb_distances (BF16 or FP8 only) and
 * also, into ws, the smallest value of every whole group of 16 consecutive
 * entries of each row; emb_topk_groups then gives exactly what emb_topk_min
 * gives for that D, but bounds the k smallest from the group minima (1/16 of
 * D's bytes) and reads only the groups that can hold them. Where k is too
 * large for the bound (more than 8 per full chunk of 2,048 entries) it selects
 * each row with one block. ws must not change between the two calls, which
 * take the same M and N; DB_ENOSPC if ws is missing or too small. */
size_t emb_groups_workspace_bytes(int M, int N);
int emb_distances_groups(int fmt, int M, int N, int dim, const void *q_codes,
                         const float *q_scale, const float *q_sq, const void *x_codes,
                         const float *x_scale, const float *x_sq, float *D, void *ws,
                         size_t ws_bytes, void *stream);
int emb_topk_groups(int M, int N, const float *D, int k, int32_t *idx, float *d, void *ws,
                    size_t ws_bytes, void *stream);

/* The k nearest database latents of each query in one pass, without a distance
 * matrix in memory: idx [M][k] (int32, device) holds, per query row, the k
 * smallest expanded-form distances of emb_distances in ascending order, ties
 * by lower index -- exactly what emb_topk_min returns for those distances.
 * d [M][k] (float, device): with direct = 0 those same expanded-form values;
 * with direct != 0 the direct form sum_i (q_i - x_i)^2 of each selected pair,
 * over the stored (dequantised) values, summed in float64 and rounded once to
 * float (within 2^-24 relative of the float64 value; exactly 0 for identical
 * codes and scales). BF16 or FP8 only; 1 <= k <= min(N, 256); ws (device,
 * 256-byte aligned) of emb_knn_workspace_bytes bytes; query codes below 2 GiB
 * and database codes below 4 GiB (DB_EINVAL otherwise); other argument rules as
 * emb_distances. */
size_t emb_knn_workspace_bytes(int M, int N, int k);
int emb_knn(int fmt, int M, int N, int dim, const void *q_codes, const float *q_scale,
            const float *q_sq, const void *x_codes, const float *x_scale, const float *x_sq, int k,
            int direct, int32_t *idx, float *d, void *ws, size_t ws_bytes, void *stream);

/* Exact re-scoring: for query q (labels [nq][nz][ny][nx]) and its candidate
 * entries cand [nq][nc] (device int32, each in [0, db_size())), the k best by
 * Dice_T1Gd + Dice_FLAIR (score desc, index asc) among the candidates.
 * nc <= DB_KMAX, k <= nc. Candidates must be distinct within a row. Each
 * overlap is counted over the x-rows inside both sides' boxes of that mask
 * (the FLAIR overlap inside both row boxes, the T1Gd one inside both T1Gd
 * boxes): every other row is zero on one side. With the block counts kept
 * (bcnt above), k <= 64 and nc > n1 = max(16, k) rounded up to 16, the
 * candidates are scored in decreasing order of a bound on their score (the
 * score formula at the sums over 16^3 blocks of the smaller of the two
 * sides' counts, which no overlap exceeds): the first n1, then only those
 * whose bound reaches the k-th best of those n1 scores. Every candidate left
 * out scores below that, so the top k are the same, bit for bit, as when
 * scoring them all (db_set_rerank_bound). */
size_t db_rerank_workspace_bytes(const db_t *db, int nq);
int db_rerank(const db_t *db, int nq, const uint8_t *q_labels, const int32_t *cand, int nc, int k,
              int32_t *idx, double *score, db_counts_t *counts, void *ws, size_t ws_bytes,
              void *stream);

/* db_rerank in two calls, so the packing of the queries (one read of their
 * labels) can run on another stream while the candidates are being found:
 * db_rerank_pack writes the queries' bit planes, mask counts and row boxes into
 * ws; db_rerank_packed then scores cand against them. Same ws (same nq, at
 * least db_rerank_workspace_bytes(db, nq) bytes, 256-byte aligned) for both
 * calls; the second must be ordered after the first (same stream, or an event).
 * Results equal db_rerank's bit for bit. Argument rules as db_rerank's.
 * After db_rerank_pack, ws begins with the queries' packed masks, uint32
 * [nq][2][Wp] in the database's plane layout (LSB-first, x fastest; plane 0
 * FLAIR, plane 1 T1Gd; Wp = nx ny nz / 32 rounded up to a multiple of 4),
 * which nn_pool_conv_planes can encode without reading the labels again. */
int db_rerank_pack(const db_t *db, int nq, const uint8_t *q_labels, void *ws, size_t ws_bytes,
                   void *stream);
/* db_rerank_pack that also writes, from the same single read of the labels, the input of
 * the encoder's first layer (Sec. 2.3, "Autoencoders": the masks mean-pooled by 2 in each
 * direction): pooled (device uint8 [nq][nz/2][ny/2][nx/2], 8-byte aligned, written whole)
 * holds per 2x2x2 block of voxels its FLAIR count (0..8) in bits 0..3 and its T1Gd count
 * (0..8) in bits 4..7; the pooled masks are those counts / 8, and nn_pool_conv_counts_bf16
 * encodes them. ws as after db_rerank_pack, bit for bit. DB_EINVAL when ny or nz is odd or
 * pooled is NULL / misaligned; other rules as db_rerank_pack. */
int db_rerank_pack_pool(const db_t *db, int nq, const uint8_t *q_labels, uint8_t *pooled,
                        void *ws, size_t ws_bytes, void *stream);
int db_rerank_packed(const db_t *db, int nq, const int32_t *cand, int nc, int k, int32_t *idx,
                     double *score, db_counts_t *counts, void *ws, size_t ws_bytes, void *stream);

/* The chain distances -> n_cand nearest latents -> exact rerank -> k best.
 * Database latents x_* have n_lat = db_size() rows. cand_idx / cand_d [nq][n_cand]
 * receive the latent candidates (or pass NULL to keep them in the workspace):
 * the n_cand nearest by expanded-form distance (ties by index), and for BF16 /
 * FP8 with n_cand <= 256 (the emb_knn path, no distance matrix) their direct-
 * form distances as emb_knn(direct = 1) reports them; otherwise (binary codes,
 * larger n_cand) the distances the selection ranked. */
size_t db_query_embed_workspace_bytes(const db_t *db, int nq, int n_cand);
int db_query_embed(const db_t *db, int fmt, int nq, int dim, const void *q_codes,
                   const float *q_scale, const float *q_sq, const void *x_codes,
                   const float *x_scale, const float *x_sq, const uint8_t *q_labels, int n_cand,
                   int k, int32_t *idx, double *score, db_counts_t *counts, int32_t *cand_idx,
                   float *cand_d, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------- centre-of-mass prefilter --- */
/* The location step of the paper's radiomics query (Sec. 2.3): keep the
 * n_cand entries whose FLAIR centre of mass is nearest the query's, then
 * score those exactly with Dice_T1Gd + Dice_FLAIR and return the k best (the
 * paper ranks its 1,000 candidates by shape features instead; exact Dice is
 * this library's choice). Key: squared distance of the centres, computed in
 * double (centre = moment / count) and rounded once to float; ties by index;
 * an empty FLAIR mask on either side gives +inf. q_labels: device uint8
 * [nq][nz][ny][nx]; outputs idx [nq][k], score [nq][k], counts [nq][k] or
 * NULL, cand_idx [nq][n_cand] or NULL, cand_d [nq][n_cand] or NULL (device).
 * 1 <= k <= n_cand <= min(db_size(), DB_KMAX), nq <= 65535. */
size_t db_query_com_workspace_bytes(const db_t *db, int nq, int n_cand);
int db_query_com(const db_t *db, int nq, const uint8_t *q_labels, int n_cand, int k, int32_t *idx,
                 double *score, db_counts_t *counts, int32_t *cand_idx, float *cand_d, void *ws,
                 size_t ws_bytes, void *stream);

/* ------------------------------------------------- downsampled queries --- */
/* The paper's cheaper exact variant (Sec. 2.3, DS64 / DS32 in Tables 1-2):
 * downsample database and query by order-0 (nearest-neighbour) spline
 * interpolation and run the same Dice query at the lower resolution. Output
 * voxel o of an axis reads source voxel round(o (n_in - 1) / (n_out - 1)).
 * Output axes are 1..256 voxels (dst nx % 32 == 0 as for any database). */

/* Append entries [first, first + n) of src to dst, resampled to dst's grid
 * (thresholds must match). The masks are resampled directly: thresholding
 * commutes with order-0 sampling. Fills dst's box and moments too. */
int db_append_resampled(db_t *dst, const db_t *src, int64_t first, int64_t n, void *stream);

/* Resample nq query label volumes uint8 [nq][nz][ny][nx] to [nq][mz][my][mx] (device). */
int labels_resample(int nq, const uint8_t *in, int nx, int ny, int nz, uint8_t *out, int mx,
                    int my, int mz, void *stream);

/* ----------------------------------------------------------------- misc --- */

/* Wait for `stream` and report any asynchronous device error as DB_EHIP. */
int db_sync(const db_t *db, void *stream);

/* Timing of the dominant kernel: while enabled, every db_scan / db_query /
 * db_query_sparse records a HIP event pair on its stream around the overlap-
 * scan kernel, every db_rerank / db_query_embed / db_query_com one around the
 * candidate-scoring kernel and every db_query_batch one around its graph
 * launch. db_profile_read waits
 * for the recorded events, returns their summed elapsed milliseconds and the
 * number of pairs, and clears them. For measurement, not for production. */
int db_profile(db_t *db, int enable);
int db_profile_read(db_t *db, double *ms, int64_t *launches);

/* Release the handle (host memory only; the storage belongs to the caller).
 * Waits for no stream: the caller must not free storage still in use. */
void db_free(db_t *db);

/* Message of the last failing call on this thread ("" if none). Valid until
 * the next library call on the same thread. */
const char *db_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TUMORDB_H */
