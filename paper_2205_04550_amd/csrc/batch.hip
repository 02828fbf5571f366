// batch.hip — many queries, each restricted to its own box, in one persistent launch.
//
// Same overlap as the single-query scan (paper Sec. 2.3: Dice of both masks,
// summed), but query q only looks at voxels inside its box R_q, on both
// sides: I_m = |A_m n B_m n R_q|, and the database side's |B_m n R_q| is
// counted on the fly (it depends on the box). The query words were ROI-masked
// when packed, so only the database side needs the x-edge masks.
//
// Work: item = (query q, tile of kTile consecutive entries). Items are held
// in 8 queues, one per XCD: queue x owns tiles t = x, x+8, ... and, inside a
// tile, the queries in descending cost order (cost = box words). Workgroups
// are dispatched round-robin over the XCDs, so block b starts on queue b % 8
// and the tiles a queue touches stay in that XCD's L2 while every query
// passes over them. A block that finds its queue empty steals from the
// others, so every item is done even if the dispatch order differs; the
// mapping only affects speed. Every block exits once all 8 queues are empty.
#include "common.hpp"
#include "internal.hpp"

namespace tdb {

constexpr int kTile = 4;
constexpr int kXcd = 8;

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

__global__ void __launch_bounds__(256) batch_scan_kernel(
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

hipError_t launch_batch_scan(const db_t *db, int64_t n, int nq, const uint32_t *qpack,
                             const int32_t *rois, const int32_t *plan, int64_t n_items,
                             int32_t *counters, uint32_t *inter, uint32_t *bcnt, hipStream_t s)
{
    (void)n_items;
    const Geometry &g = db->g;
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int blocks = db->cus * 8;
    hipLaunchKernelGGL(batch_scan_kernel, dim3(blocks), dim3(256), 0, s, db->planes, g.Wp, g.nxw,
                       g.ny, n, nq, qpack, rois, plan, ntiles, counters, inter, bcnt,
                       2 * db->capacity);
    return hipGetLastError();
}

}  // namespace tdb
