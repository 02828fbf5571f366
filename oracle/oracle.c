/*
 * oracle.c — plain, slow, obviously correct CPU oracle of the retrieval scan.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. The GPU product path never calls it.
 * It shares no code, header or constant with the GPU library: it works voxel
 * by voxel on unpacked values (no bit packing, no popcount).
 *
 * What it follows (A for-loop is all you need, arXiv 2205.04550):
 *   - Sec. 2.3 "Query to a database": each simulation is thresholded into a
 *     FLAIR mask (lower threshold) and a T1Gd mask (higher threshold).
 *   - Sec. 2.3: the Dice coefficient is the similarity measure.
 *   - Sec. 2.3: the two similarities are added, Dice_T1Gd + Dice_FLAIR, and
 *     the highest sum is the best match.
 *   - Sec. 2.3 "Baseline for-loop search": the ground truth is a plain loop
 *     over the database comparing the query with every entry.
 *
 * Readings where the paper is silent (each pinned by a test):
 *   - a voxel belongs to a mask when c >= t (float32 compare);
 *   - Dice(empty, empty) = 1; Dice = 2|A n B| / (|A| + |B|) in IEEE double;
 *   - an optional half-open box ROI restricts both masks (not in the paper);
 *   - ranking is by (score descending, index ascending) — done by the Python
 *     side with a full sort.
 */
#include <stdint.h>
#include <stdlib.h>

/* L[v] = (c[v] >= t_lo) | (c[v] >= t_hi) << 1 : bit0 FLAIR, bit1 T1Gd. */
void oracle_threshold(const float *c, int64_t nvox, float t_lo, float t_hi, uint8_t *L)
{
    for (int64_t v = 0; v < nvox; ++v) {
        uint8_t flair = (c[v] >= t_lo) ? 1 : 0;
        uint8_t t1 = (c[v] >= t_hi) ? 1 : 0;
        L[v] = (uint8_t)(flair | (t1 << 1));
    }
}

/*
 * Overlap counts of query labels q and database labels L inside the box
 * roi = {x0, y0, z0, x1, y1, z1} (half-open; NULL = whole grid).
 * out = {I_FLAIR, I_T1, A_FLAIR, A_T1, B_FLAIR, B_T1} where for mask m
 *   I_m = #{v in R : a_m(v) and b_m(v)},  A_m = #{v in R : a_m(v)},
 *   B_m = #{v in R : b_m(v)},  a_m(v) = bit m of q[v], b_m(v) = bit m of L[v].
 */
void oracle_counts(const uint8_t *q, const uint8_t *L, int nx, int ny, int nz,
                   const int32_t *roi, uint64_t out[6])
{
    int x0 = 0, y0 = 0, z0 = 0, x1 = nx, y1 = ny, z1 = nz;
    if (roi) {
        x0 = roi[0]; y0 = roi[1]; z0 = roi[2];
        x1 = roi[3]; y1 = roi[4]; z1 = roi[5];
    }
    uint64_t I[2] = {0, 0}, A[2] = {0, 0}, B[2] = {0, 0};
    for (int z = z0; z < z1; ++z)
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                int64_t v = ((int64_t)z * ny + y) * nx + x;
                for (int m = 0; m < 2; ++m) {
                    unsigned a = (q[v] >> m) & 1u;
                    unsigned b = (L[v] >> m) & 1u;
                    I[m] += a & b;
                    A[m] += a;
                    B[m] += b;
                }
            }
    out[0] = I[0];
    out[1] = I[1];
    out[2] = A[0];
    out[3] = A[1];
    out[4] = B[0];
    out[5] = B[1];
}

/* Dice = 2I / (A + B) in IEEE double; 1 when both masks are empty. */
double oracle_dice(uint64_t I, uint64_t A, uint64_t B)
{
    if (A + B == 0)
        return 1.0;
    return (double)(2 * I) / (double)(A + B);
}

/* Summed score of one entry: Dice_T1Gd + Dice_FLAIR. */
double oracle_score(const uint64_t cnt[6])
{
    double d_flair = oracle_dice(cnt[0], cnt[2], cnt[4]);
    double d_t1 = oracle_dice(cnt[1], cnt[3], cnt[5]);
    return d_t1 + d_flair;
}

/*
 * The for-loop over a block of database entries: threshold entry n's
 * concentration volume, count against the query, store counts[n][6] and
 * score[n]. Entries are independent, so the loop is split over threads.
 */
void oracle_scan_block(const float *conc, int64_t n, int nx, int ny, int nz, float t_lo,
                       float t_hi, const uint8_t *q, const int32_t *roi, uint64_t *counts,
                       double *score, int nthreads)
{
    int64_t V = (int64_t)nx * ny * nz;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        uint8_t *L = (uint8_t *)malloc((size_t)V);
        if (!L)
            abort();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            oracle_threshold(conc + i * V, V, t_lo, t_hi, L);
            oracle_counts(q, L, nx, ny, nz, roi, counts + 6 * i);
            score[i] = oracle_score(counts + 6 * i);
        }
        free(L);
    }
}

/*
 * The same for-loop with several queries: entry n is thresholded once and then
 * counted against each query j (labels q + j*V, box rois + 6j, or the whole grid
 * when rois is NULL). counts[j][n][6], score[j][n].
 */
void oracle_scan_block_multi(const float *conc, int64_t n, int nx, int ny, int nz, float t_lo,
                             float t_hi, int nq, const uint8_t *q, const int32_t *rois,
                             uint64_t *counts, double *score, int nthreads)
{
    int64_t V = (int64_t)nx * ny * nz;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        uint8_t *L = (uint8_t *)malloc((size_t)V);
        if (!L)
            abort();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            oracle_threshold(conc + i * V, V, t_lo, t_hi, L);
            for (int j = 0; j < nq; ++j) {
                uint64_t *c = counts + 6 * ((int64_t)j * n + i);
                oracle_counts(q + (int64_t)j * V, L, nx, ny, nz, rois ? rois + 6 * j : NULL, c);
                score[(int64_t)j * n + i] = oracle_score(c);
            }
        }
        free(L);
    }
}
