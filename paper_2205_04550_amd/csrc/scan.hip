// scan.hip — the exhaustive overlap scan of one query against every database entry.
//
// Paper Sec. 2.3, "Baseline for-loop search": compare the query with every
// database tumour; entries are independent, so the loop is parallel. For
// bit-packed masks the Dice numerator of mask m of entry n is
//     I_m(n) = sum_w popcount(Q_m[w] & D_m(n)[w]),
// and the database side's |B_m(n)| was stored at build time. The scan is a
// pure stream of the packed database (2 * V / 8 bytes per entry) through
// AND + popcount: HBM-bound by design.
//
// Mapping: one 256-thread block per SIMS consecutive entries; every thread
// reads 16-byte words of both mask planes with non-temporal loads, UNROLL
// deep, so each wave keeps UNROLL * SIMS * 2 KiB of loads in flight. The
// query (2 * Wp words) is re-read from L2 by every block and amortised over
// the SIMS entries of the block. SIMS = 2, UNROLL = 2 was the fastest of a
// sweep over block size (256/512/1024), SIMS (1/2/4), UNROLL (2/4/8),
// persistent vs one-shot grids and temporal vs non-temporal loads: 6.99 TB/s
// against 7.13-7.17 TB/s for a plain non-temporal read of the same bytes;
// SIMS = 1 loses ~10% to the doubled L2 traffic of the query.
#include "common.hpp"
#include "internal.hpp"

namespace tdb {

template <int SIMS, int UNROLL, bool TAIL>
__global__ void __launch_bounds__(256) scan_kernel(const u32x4 *__restrict__ db, int64_t rec_u4,
                                                   int plane_u4, const u32x4 *__restrict__ q,
                                                   int64_t n, uint32_t *__restrict__ inter)
{
    __shared__ uint32_t red[SIMS][2 * 4];
    const int64_t e0 = (int64_t)blockIdx.x * SIMS;
    uint32_t c0[SIMS], c1[SIMS];
    const u32x4 *d[SIMS];
#pragma unroll
    for (int s = 0; s < SIMS; ++s) {
        c0[s] = 0;
        c1[s] = 0;
        // Entries past n alias the last valid one; their counts are discarded.
        const int64_t e = (e0 + s < n) ? e0 + s : n - 1;
        d[s] = db + e * rec_u4;
    }
    for (int base = 0; base < plane_u4; base += 256 * UNROLL) {
        u32x4 q0[UNROLL], q1[UNROLL], v0[UNROLL][SIMS], v1[UNROLL][SIMS];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int i = base + u * 256 + threadIdx.x;
            if (!TAIL || i < plane_u4) {
                q0[u] = q[i];
                q1[u] = q[plane_u4 + i];
#pragma unroll
                for (int s = 0; s < SIMS; ++s) {
                    v0[u][s] = load_stream(d[s] + i);
                    v1[u][s] = load_stream(d[s] + plane_u4 + i);
                }
            } else {
                q0[u] = q1[u] = (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
                for (int s = 0; s < SIMS; ++s)
                    v0[u][s] = v1[u][s] = (u32x4){0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int s = 0; s < SIMS; ++s) {
                c0[s] += popc_and4(q0[u], v0[u][s]);
                c1[s] += popc_and4(q1[u], v1[u][s]);
            }
    }
#pragma unroll
    for (int s = 0; s < SIMS; ++s) {
        block_sum2(c0[s], c1[s], red[s]);
        if (threadIdx.x == 0 && e0 + s < n) {
            inter[2 * (e0 + s)] = c0[s];
            inter[2 * (e0 + s) + 1] = c1[s];
        }
    }
}

hipError_t launch_scan(const db_t *db, int64_t n, const uint32_t *qpack, uint32_t *inter,
                       hipStream_t s)
{
    const int plane_u4 = db->g.Wp / 4;
    const int64_t rec_u4 = 2 * (int64_t)plane_u4;
    constexpr int SIMS = 2, UNROLL = 2;
    const int64_t blocks = (n + SIMS - 1) / SIMS;
    const auto *dbp = reinterpret_cast<const u32x4 *>(db->planes);
    const auto *qp = reinterpret_cast<const u32x4 *>(qpack);
    // Planes that are a whole number of block steps need no tail test.
    if (plane_u4 % (256 * UNROLL) == 0)
        hipLaunchKernelGGL((scan_kernel<SIMS, UNROLL, false>), dim3((unsigned)blocks), dim3(256),
                           0, s, dbp, rec_u4, plane_u4, qp, n, inter);
    else
        hipLaunchKernelGGL((scan_kernel<SIMS, UNROLL, true>), dim3((unsigned)blocks), dim3(256), 0,
                           s, dbp, rec_u4, plane_u4, qp, n, inter);
    return hipGetLastError();
}

}  // namespace tdb
