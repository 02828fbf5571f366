// batch.hip — many queries, each restricted to its own box, in one launch.
//
// Same overlap as the single-query scan (paper Sec. 2.3: Dice of both masks,
// summed), but query q only looks at voxels inside its box R_q, on both
// sides: I_m = |A_m n B_m n R_q|, and the database side's |B_m n R_q| is
// counted on the fly (it depends on the box). The query words were ROI-masked
// when packed, so only the database side needs x-edge masks.
//
// Main kernel (batch_lds_kernel): one block per work item (tile, query chunk).
// Tiles are groups of TILE entries (4 or 8) ordered by their cost, largest first,
// and blocks are dispatched in item order, so the long items start early and the
// short ones fill in at the end (a persistent grid taking the items from an atomic
// counter was measured 20-35 % slower). An item streams its tile's entries through
// LDS in z-slabs of Z planes, so every database word is read from HBM once per
// query chunk. For each slab, the block's waves
// take the queries whose box meets the slab (a host-built list, costliest
// first) and run them against the LDS copy: a lane per box row, the packed
// query row from L2 reused for the kTile entries. Per-(query, entry) counters
// live in LDS; a wave folds its 16 partial counters with a reduce-scatter (17
// shuffles) and adds them there; the block writes them out after the last
// slab. The work is integer VALU bound: per packed word and mask, AND +
// popcount for I and AND + popcount for |B n R|.
//
// Fallback (batch_rows_kernel): grids whose one-plane slab does not fit in LDS
// use a persistent (query, tile) kernel that reads the database through L2.
// Its items sit in 8 queues, one per XCD (tile t in queue t % 8, queries in
// descending cost inside a tile); block b starts on queue b % 8 (dispatch is
// round-robin over XCDs) and steals from the others when its queue is empty,
// so every item is done whatever the dispatch order; the mapping only affects
// L2 locality. Every block exits once all 8 queues are empty.
#include <limits.h>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace tdb {

constexpr int kTile = 4;        // entries per item of the L2 fallback kernel
constexpr int kXcd = 8;
constexpr int kBatchThreads = 1024;
constexpr int kQueryChunk = 256;   // queries whose counters share one block's LDS
constexpr int kStageBatch = 8;     // slab-staging loads in flight per thread

// ceil(2^32 / d) for d >= 2 (d = 1 is handled by the caller: it would need 2^32).
// floor(r * M / 2^32) == r / d whenever r * d < 2^32, which the host
// guarantees by requiring ny * ny * nz < 2^32.
__device__ __forceinline__ uint32_t magic_u32(uint32_t d)
{
    return (uint32_t)((0x100000000ULL + d - 1) / d);
}

__device__ __forceinline__ uint32_t div_magic(uint32_t r, uint32_t d, uint32_t M)
{
    return d == 1 ? r : __umulhi(r, M);
}

// Bits of word wx (voxels x = 32 wx .. 32 wx + 31) inside [x0, x1).
__device__ __forceinline__ uint32_t xmask(int wx, int x0, int x1)
{
    const int lo = x0 - 32 * wx, hi = x1 - 32 * wx;
    if (hi <= 0 || lo >= 32) return 0u;
    uint32_t m = 0xffffffffu;
    if (lo > 0) m &= 0xffffffffu << lo;
    if (hi < 32) m &= (1u << hi) - 1u;
    return m;
}

// Sum 16 per-lane values over the 64 lanes of a wave with 17 shuffles
// (halve the value set at each xor step, then fold the last two lane bits).
// Every lane returns the total of value number
//   ((lane >> 5) & 1) << 3 | ((lane >> 4) & 1) << 2 | ((lane >> 3) & 1) << 1 | ((lane >> 2) & 1).
__device__ __forceinline__ uint32_t reduce16(const uint32_t (&v)[16], int lane)
{
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
    uint32_t a[8], b[4], c[2];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t send = h5 ? v[j] : v[j + 8];
        const uint32_t keep = h5 ? v[j + 8] : v[j];
        a[j] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t send = h4 ? a[j] : a[j + 4];
        const uint32_t keep = h4 ? a[j + 4] : a[j];
        b[j] = keep + __shfl_xor(send, 16, 64);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const uint32_t send = h3 ? b[j] : b[j + 2];
        const uint32_t keep = h3 ? b[j + 2] : b[j];
        c[j] = keep + __shfl_xor(send, 8, 64);
    }
    const uint32_t send = h2 ? c[0] : c[1];
    const uint32_t keep = h2 ? c[1] : c[0];
    uint32_t d = keep + __shfl_xor(send, 4, 64);
    d += __shfl_xor(d, 2, 64);
    d += __shfl_xor(d, 1, 64);
    return d;
}

// Rows of 128 voxels (4 words per mask) for a box whose x-range covers words
// W0..W1: only those words are counted; the database side needs a mask only on
// the two edge words (the query side was masked when packed).
template <int TILE, int W0, int W1>
__device__ __forceinline__ void count_rows4(uint32_t (&acc)[4 * TILE], const uint32_t *D, int slab_w,
                                            const uint32_t *Q0, const uint32_t *Q1, uint32_t nr,
                                            uint32_t nyr, uint32_t M, int zlo, int y0, int zs0,
                                            int ny, uint32_t mlo, uint32_t mhi, int lane)
{
    // Two rows per lane per pass: both rows' query loads (L2) are issued before either
    // row is counted; a second row past nr loads row 0 of the box and is not counted.
    for (uint32_t r0 = lane; r0 < nr; r0 += 128) {
        u32x4 qa[2], qb[2];
        int lw[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint32_t r = r0 + 64 * u < nr ? r0 + 64 * u : 0u;
            const uint32_t zr = div_magic(r, nyr, M);
            const int z = zlo + (int)zr;
            const int y = y0 + (int)(r - zr * nyr);
            const int gw = (z * ny + y) * 4;
            lw[u] = ((z - zs0) * ny + y) * 4;
            qa[u] = *reinterpret_cast<const u32x4 *>(Q0 + gw);
            qb[u] = *reinterpret_cast<const u32x4 *>(Q1 + gw);
        }
        const bool live1 = r0 + 64 < nr;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !live1) break;
#pragma unroll
            for (int s = 0; s < TILE; ++s) {
                const u32x4 da = *reinterpret_cast<const u32x4 *>(D + (2 * s) * slab_w + lw[u]);
                const u32x4 db = *reinterpret_cast<const u32x4 *>(D + (2 * s + 1) * slab_w + lw[u]);
#pragma unroll
                for (int w = W0; w <= W1; ++w) {
                    const uint32_t dwa = da[w], dwb = db[w];
                    acc[4 * s + 0] = popc_acc(qa[u][w] & dwa, acc[4 * s + 0]);
                    acc[4 * s + 1] = popc_acc(qb[u][w] & dwb, acc[4 * s + 1]);
                    if (w == W0 || w == W1) {
                        const uint32_t m = (W0 == W1) ? (mlo & mhi) : (w == W0 ? mlo : mhi);
                        acc[4 * s + 2] = popc_acc(dwa & m, acc[4 * s + 2]);
                        acc[4 * s + 3] = popc_acc(dwb & m, acc[4 * s + 3]);
                    } else {
                        acc[4 * s + 2] = popc_acc(dwa, acc[4 * s + 2]);
                        acc[4 * s + 3] = popc_acc(dwb, acc[4 * s + 3]);
                    }
                }
            }
        }
    }
}

// grid = ntiles * nchunks blocks, kBatchThreads (or the tuned block size) threads.
// Dynamic LDS:
//   D   uint32 [TILE][2][Z * ny * nxw]    the tile's slab, both masks
//   cnt uint32 [qchunk][TILE][4]          I_FLAIR, I_T1Gd, |B_FLAIR n R|, |B_T1Gd n R|
// Block i does item i: tile i / nchunks and query chunk i % nchunks. list_off [nchunks * nslabs + 1] / list_q: per (chunk,
// slab) the queries whose box meets the slab.
//
// Tile t holds entries tile_order[TILE t .. TILE t + TILE - 1] (entries sorted by the
// centre of their stored row boxes, so a tile's members overlap; tiles ordered by the
// size of the union of their members' row boxes, largest first). Rows outside that
// union are zero in every member and add nothing to I or |B n R|: slabs outside it are
// neither staged nor scanned, and each query's rows are clipped to it.
template <int TILE>
__global__ void __launch_bounds__(kBatchThreads) batch_lds_kernel(
    const uint32_t *__restrict__ planes, int Wp, int nxw, int ny, int nz, int64_t n, int Z,
    int nslabs, const uint32_t *__restrict__ qpack, const int32_t *__restrict__ rois,
    const int32_t *__restrict__ list_off, const int32_t *__restrict__ list_q, int qchunk, int nq,
    int nchunks, const int32_t *__restrict__ tile_order,
    const int32_t *__restrict__ ebox, uint32_t *__restrict__ inter, uint32_t *__restrict__ bcnt,
    int64_t out_qstride)
{
    extern __shared__ u32x4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    const int plane_w = ny * nxw;              // words per z-plane of one mask
    const int slab_w = Z * plane_w;            // words per slab of one mask
    uint32_t *D = lds;                         // [TILE][2][slab_w]
    uint32_t *cnt = lds + TILE * 2 * slab_w;   // [qchunk][TILE][4]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    {
        const int64_t item = blockIdx.x;
        const int64_t tile = item / nchunks;
        const int chunk = (int)(item - tile * nchunks);
        const int q0 = chunk * qchunk;
        const int nqc = min(qchunk, nq - q0);
        const int64_t e0 = tile * TILE;

        for (int i = threadIdx.x; i < nqc * TILE * 4; i += blockDim.x)
            cnt[i] = 0;
        // The tile's members and the union of their row boxes.
        int64_t ent[TILE];
        int uz0 = INT_MAX, uz1 = INT_MIN, uy0 = INT_MAX, uy1 = INT_MIN;
#pragma unroll
        for (int s = 0; s < TILE; ++s) {
            const int64_t p = (e0 + s < n) ? e0 + s : n - 1;   // alias past the end
            ent[s] = tile_order ? (int64_t)tile_order[p] : p;
            const int32_t *b = ebox + 4 * ent[s];
            if (b[1] > b[0] && b[3] > b[2]) {
                uz0 = min(uz0, b[0]);
                uz1 = max(uz1, b[1]);
                uy0 = min(uy0, b[2]);
                uy1 = max(uy1, b[3]);
            }
        }

        for (int slab = 0; slab < nslabs; ++slab) {
            const int zs0 = slab * Z;
            const int zn = min(Z, nz - zs0);
            const int words = zn * plane_w;
            if (zs0 >= uz1 || zs0 + zn <= uz0) continue;   // block-uniform: no member has a row here
            __syncthreads();  // the previous slab is consumed; counters are zeroed
            // Stage the tile's slab: TILE entries x 2 masks x `words` words.
            if ((plane_w & 3) == 0) {
                // kStageBatch loads per thread in flight before any is stored.
                const int w4 = words >> 2;
                const int tot = TILE * 2 * w4;
                for (int i0 = threadIdx.x; i0 < tot; i0 += kStageBatch * blockDim.x) {
                    u32x4 v[kStageBatch];
                    int dst[kStageBatch];
#pragma unroll
                    for (int u = 0; u < kStageBatch; ++u) {
                        const int i = i0 + u * blockDim.x;
                        const int sm = i / w4;
                        const int j = i - sm * w4;
                        const int s = sm >> 1, m = sm & 1;
                        dst[u] = -1;
                        if (i < tot) {
                            const int64_t e = ent[s & (TILE - 1)];
                            const u32x4 *g = reinterpret_cast<const u32x4 *>(
                                planes + e * 2 * (int64_t)Wp + (int64_t)m * Wp +
                                (int64_t)zs0 * plane_w);
                            v[u] = load_stream(g + j);
                            dst[u] = sm * (slab_w >> 2) + j;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kStageBatch; ++u)
                        if (dst[u] >= 0) reinterpret_cast<u32x4 *>(D)[dst[u]] = v[u];
                }
            } else {
                for (int i = threadIdx.x; i < TILE * 2 * words; i += blockDim.x) {
                    const int sm = i / words;
                    const int j = i - sm * words;
                    const int s = sm >> 1, m = sm & 1;
                    const int64_t e = ent[s];
                    D[sm * slab_w + j] =
                        planes[e * 2 * (int64_t)Wp + (int64_t)m * Wp + (int64_t)zs0 * plane_w + j];
                }
            }
            __syncthreads();
            const int lo = list_off[chunk * nslabs + slab];
            const int hi = list_off[chunk * nslabs + slab + 1];
            for (int li = lo + wave; li < hi; li += nwaves) {
                const int q = list_q[li];
                const int32_t *R = rois + 6 * q;
                const int x0 = R[0], x1 = R[3];
                const int y0 = max(R[1], uy0), y1 = min(R[4], uy1);
                const int zlo = max(max(R[2], zs0), uz0), zhi = min(min(R[5], zs0 + zn), uz1);
                const uint32_t nyr = y1 > y0 ? (uint32_t)(y1 - y0) : 0u;
                const uint32_t nr = (zhi > zlo) ? (uint32_t)(zhi - zlo) * nyr : 0u;
                const uint32_t M = nyr > 1 ? magic_u32(nyr) : 0u;
                const uint32_t *Q0 = qpack + (int64_t)q * 2 * Wp;
                const uint32_t *Q1 = Q0 + Wp;
                uint32_t acc[4 * TILE];
#pragma unroll
                for (int j = 0; j < 4 * TILE; ++j) acc[j] = 0;
                if (nxw == 4) {
                    // 128-voxel rows: one 16-byte word group per row and mask, counted
                    // over the box's words only (10 word ranges, each its own loop).
                    const int wx0 = x0 >> 5, wx1 = (x1 - 1) >> 5;
                    const uint32_t mlo = 0xffffffffu << (x0 & 31);
                    const uint32_t mhi = (x1 & 31) ? ((1u << (x1 & 31)) - 1u) : 0xffffffffu;
#define TDB_ROWS(a, b)                                                                          \
    count_rows4<TILE, a, b>(acc, D, slab_w, Q0, Q1, nr, nyr, M, zlo, y0, zs0, ny, mlo, mhi, lane)
                    switch (wx0 * 4 + wx1) {
                    case 0: TDB_ROWS(0, 0); break;
                    case 1: TDB_ROWS(0, 1); break;
                    case 2: TDB_ROWS(0, 2); break;
                    case 3: TDB_ROWS(0, 3); break;
                    case 5: TDB_ROWS(1, 1); break;
                    case 6: TDB_ROWS(1, 2); break;
                    case 7: TDB_ROWS(1, 3); break;
                    case 10: TDB_ROWS(2, 2); break;
                    case 11: TDB_ROWS(2, 3); break;
                    default: TDB_ROWS(3, 3); break;
                    }
#undef TDB_ROWS
                } else {
                    const int wx0 = x0 >> 5, wx1 = (x1 - 1) >> 5;
                    for (uint32_t r = lane; r < nr; r += 64) {
                        const uint32_t zr = div_magic(r, nyr, M);
                        const int z = zlo + (int)zr;
                        const int y = y0 + (int)(r - zr * nyr);
                        const int gw = (z * ny + y) * nxw;
                        const int lw = ((z - zs0) * ny + y) * nxw;
                        for (int wx = wx0; wx <= wx1; ++wx) {
                            const uint32_t xm = xmask(wx, x0, x1);
                            const uint32_t qa = Q0[gw + wx], qb = Q1[gw + wx];
#pragma unroll
                            for (int s = 0; s < TILE; ++s) {
                                const uint32_t da = D[(2 * s) * slab_w + lw + wx];
                                const uint32_t db = D[(2 * s + 1) * slab_w + lw + wx];
                                acc[4 * s + 0] += popc(qa & da);
                                acc[4 * s + 1] += popc(qb & db);
                                acc[4 * s + 2] += popc(da & xm);
                                acc[4 * s + 3] += popc(db & xm);
                            }
                        }
                    }
                }
                // Fold the lanes' counters 16 at a time (four entries per group).
#pragma unroll
                for (int g = 0; g < TILE / 4; ++g) {
                    uint32_t part[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) part[j] = acc[16 * g + j];
                    const uint32_t tot = reduce16(part, lane);
                    if ((lane & 3) == 0) {
                        const int vidx = (((lane >> 5) & 1) << 3) | (((lane >> 4) & 1) << 2) |
                                         (((lane >> 3) & 1) << 1) | ((lane >> 2) & 1);
                        atomicAdd(&cnt[(q - q0) * TILE * 4 + 16 * g + vidx], tot);
                    }
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nqc * TILE; i += blockDim.x) {
            const int qi = i / TILE, s = i - qi * TILE;
            const int64_t e = ent[s];
            if (e0 + s < n) {
                const uint32_t *c = cnt + i * 4;
                uint32_t *io = inter + (int64_t)(q0 + qi) * out_qstride + 2 * e;
                uint32_t *bo = bcnt + (int64_t)(q0 + qi) * out_qstride + 2 * e;
                io[0] = c[0];
                io[1] = c[1];
                bo[0] = c[2];
                bo[1] = c[3];
            }
        }
    }
}

__global__ void __launch_bounds__(256) batch_rows_kernel(
    const uint32_t *__restrict__ planes, int Wp, int nxw, int ny, int64_t n, int nq,
    const uint32_t *__restrict__ qpack, const int32_t *__restrict__ rois,
    const int32_t *__restrict__ order, int64_t ntiles, int32_t *counters,
    uint32_t *__restrict__ inter, uint32_t *__restrict__ bcnt, int64_t out_qstride)
{
    __shared__ uint32_t red[2 * kTile][2 * 4];
    __shared__ int64_t s_item;
    const int home = blockIdx.x % kXcd;
    int probe = 0;  // queues tried in order home, home+1, ...
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t item = -1;
            while (probe < kXcd) {
                const int x = (home + probe) % kXcd;
                const int64_t tiles_x = (ntiles > x) ? (ntiles - x + kXcd - 1) / kXcd : 0;
                const int64_t len = tiles_x * nq;
                const int64_t i = (int64_t)atomicAdd(&counters[x], 1);
                if (i < len) {
                    const int64_t t = x + (int64_t)kXcd * (i / nq);
                    item = t * nq + order[i % nq];
                    break;
                }
                ++probe;
            }
            s_item = item;
        }
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item < 0)
            return;
        const int q = (int)(item % nq);
        const int64_t t = item / nq;
        const int32_t *R = rois + 6 * q;
        const int x0 = R[0], y0 = R[1], z0 = R[2], x1 = R[3], y1 = R[4], z1 = R[5];
        const int wx0 = x0 >> 5, wx1 = (x1 - 1) >> 5, nw = wx1 - wx0 + 1;
        const uint32_t mlo = 0xffffffffu << (x0 & 31);
        const uint32_t mhi = (x1 & 31) ? ((1u << (x1 & 31)) - 1u) : 0xffffffffu;
        const uint32_t nyr = (uint32_t)(y1 - y0);
        const uint32_t nr = (uint32_t)(z1 - z0) * nyr;
        const uint32_t M = nyr > 1 ? magic_u32(nyr) : 0u;
        const uint32_t *Q0 = qpack + (int64_t)q * 2 * Wp;
        const uint32_t *Q1 = Q0 + Wp;
        const uint32_t *D[kTile];
        const int64_t e0 = t * kTile;
#pragma unroll
        for (int s = 0; s < kTile; ++s) {
            const int64_t e = (e0 + s < n) ? e0 + s : n - 1;
            D[s] = planes + e * 2 * (int64_t)Wp;
        }
        uint32_t I0[kTile], I1[kTile], B0[kTile], B1[kTile];
#pragma unroll
        for (int s = 0; s < kTile; ++s)
            I0[s] = I1[s] = B0[s] = B1[s] = 0;
        for (uint32_t r = threadIdx.x; r < nr; r += blockDim.x) {
            const uint32_t zr = div_magic(r, nyr, M);
            const int z = z0 + (int)zr;
            const int y = y0 + (int)(r - zr * nyr);
            const int64_t base = ((int64_t)z * ny + y) * nxw + wx0;
            for (int j = 0; j < nw; ++j) {
                uint32_t xm = 0xffffffffu;
                if (j == 0) xm &= mlo;
                if (j == nw - 1) xm &= mhi;
                const uint32_t q0 = Q0[base + j], q1 = Q1[base + j];
#pragma unroll
                for (int s = 0; s < kTile; ++s) {
                    const uint32_t d0 = D[s][base + j];
                    const uint32_t d1 = D[s][Wp + base + j];
                    I0[s] += popc(q0 & d0);
                    I1[s] += popc(q1 & d1);
                    B0[s] += popc(d0 & xm);
                    B1[s] += popc(d1 & xm);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kTile; ++s) {
            block_sum2(I0[s], I1[s], red[2 * s]);
            block_sum2(B0[s], B1[s], red[2 * s + 1]);
            if (threadIdx.x == 0 && e0 + s < n) {
                uint32_t *io = inter + q * out_qstride + 2 * (e0 + s);
                uint32_t *bo = bcnt + q * out_qstride + 2 * (e0 + s);
                io[0] = I0[s];
                io[1] = I1[s];
                bo[0] = B0[s];
                bo[1] = B1[s];
            }
        }
    }
}

int batch_tile(const db_t *db) { return db->batch_tile == 8 ? 8 : 4; }

template <int TILE>
static const void *lds_kernel_ptr()
{
    return reinterpret_cast<const void *>(&batch_lds_kernel<TILE>);
}

BatchPlan batch_plan(const db_t *db, int nq)
{
    BatchPlan p{};
    const Geometry &g = db->g;
    const int tile = batch_tile(db);
    const int qc = db->batch_qchunk > 0 ? db->batch_qchunk : kQueryChunk;
    p.tile = tile;
    p.qchunk = nq < qc ? nq : qc;
    p.nchunks = (nq + p.qchunk - 1) / p.qchunk;
    const int64_t plane_bytes = (int64_t)g.ny * g.nxw * 4;
    const int64_t cnt_bytes = (int64_t)p.qchunk * tile * 4 * 4;
    const int64_t budget = (int64_t)db->lds_max - cnt_bytes;
    int64_t Z = budget > 0 ? budget / (tile * 2 * plane_bytes) : 0;
    if (db->batch_planes > 0 && db->batch_planes < Z) Z = db->batch_planes;  // tuned depth
    if (db->batch_planes < 0) Z = 0;                                           // L2 kernel forced
    if (Z > g.nz) Z = g.nz;
    p.threads = db->batch_threads > 0 ? db->batch_threads : kBatchThreads;
    p.Z = (int)Z;
    p.use_lds = Z >= 1;
    p.nslabs = p.use_lds ? (g.nz + p.Z - 1) / p.Z : 0;
    p.lds_bytes = p.use_lds ? (size_t)(tile * 2 * plane_bytes * Z + cnt_bytes) : 0;
    return p;
}

hipError_t batch_set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute(lds_kernel_ptr<4>(),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(lds_kernel_ptr<8>(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes);
    return e;
}

hipError_t launch_batch_scan(const db_t *db, int64_t n, int nq, const BatchPlan &p,
                             const uint32_t *qpack, const int32_t *rois, const int32_t *order,
                             const int32_t *list_off, const int32_t *list_q, int32_t *counters,
                             uint32_t *inter, uint32_t *bcnt, hipStream_t s)
{
    const Geometry &g = db->g;
    if (p.use_lds) {
        const int32_t *tile_order =
            db->tile_order_n == n && db->tile_order_tile == p.tile ? db->tile_order : nullptr;
        const unsigned grid = (unsigned)(((n + p.tile - 1) / p.tile) * p.nchunks);
        if (p.tile == 8)
            hipLaunchKernelGGL(batch_lds_kernel<8>, dim3(grid), dim3(p.threads), p.lds_bytes, s,
                               db->planes, g.Wp, g.nxw, g.ny, g.nz, n, p.Z, p.nslabs, qpack, rois,
                               list_off, list_q, p.qchunk, nq, p.nchunks, tile_order,
                               db->box, inter, bcnt, 2 * db->capacity);
        else
            hipLaunchKernelGGL(batch_lds_kernel<4>, dim3(grid), dim3(p.threads), p.lds_bytes, s,
                               db->planes, g.Wp, g.nxw, g.ny, g.nz, n, p.Z, p.nslabs, qpack, rois,
                               list_off, list_q, p.qchunk, nq, p.nchunks, tile_order,
                               db->box, inter, bcnt, 2 * db->capacity);
    } else {
        const int64_t ntiles = (n + kTile - 1) / kTile;
        hipLaunchKernelGGL(batch_rows_kernel, dim3(db->cus * 8), dim3(256), 0, s, db->planes, g.Wp,
                           g.nxw, g.ny, n, nq, qpack, rois, order, ntiles, counters, inter, bcnt,
                           2 * db->capacity);
    }
    return hipGetLastError();
}

}  // namespace tdb
