// sparse.hip — per-entry row boxes and mask moments, the box-restricted exact
// scan, and the centre-of-mass prefilter.
//
// Row box: the x-rows (z, y) of an entry that hold any set bit of either mask
// lie in [z0, z1) x [y0, y1). A row outside it is zero in both planes, so it
// adds nothing to I_m = sum_w popcount(Q_m[w] & D_m[w]) (Sec. 2.3, Dice), and
// neither does a row outside the query's own box. Scanning only the rows of
// the two boxes' intersection gives the same intersections, bit for bit, as
// the full scan, while reading a fraction of the bytes: a simulated tumour
// covers a small part of the atlas grid. The paper's loop reads everything;
// skipping provably-zero rows is this library's addition.
//
// Moments: sum x, sum y, sum z and the count of the FLAIR mask, exact in
// integers. Their ratio is the tumour's centre of mass, the location feature
// of the paper's radiomics query (Sec. 2.3), which keeps the 1,000 database
// entries whose centre is nearest the query's before the final comparison.
#include <float.h>

#include "common.hpp"
#include "internal.hpp"

namespace tdb {

// One 256-thread block per record of `rec_words` words (two planes of Wp words): its row box
// [4] (rows with a set bit in either mask), the row box of its T1Gd bits alone [4], its
// FLAIR moments [4] = (sum x, sum y, sum z, count) and, per z-slice, the y-range of the rows
// with a FLAIR bit and of those with a T1Gd bit (zrange [nz][2], y0 | y1 << 16, [y0, y1);
// zero when the slice has none). Boxes are [z0, z1) x [y0, y1), all zero when empty. The
// slices are taken kZChunk at a time, their ranges gathered with LDS atomics.
constexpr int kZChunk = 512;

__global__ void __launch_bounds__(256) meta_kernel(const uint32_t *__restrict__ recs,
                                                   int64_t rec_words, int Wp, int W, int nxw,
                                                   int ny, int32_t *__restrict__ box,
                                                   int32_t *__restrict__ tbox,
                                                   uint64_t *__restrict__ mom,
                                                   uint32_t *__restrict__ zrange)
{
    __shared__ int rb[4][8];
    __shared__ uint64_t rm[4][4];
    __shared__ int zy[4][kZChunk];             // per slice of the chunk: FLAIR y lo, hi; T1Gd
    const int64_t e = blockIdx.x;
    const uint32_t *P0 = recs + e * rec_words, *P1 = P0 + Wp;
    const int slice_w = ny * nxw, nz = W / slice_w;
    int bx[8] = {INT_MAX, -1, INT_MAX, -1, INT_MAX, -1, INT_MAX, -1};   // z lo/hi, y lo/hi; twice
    uint64_t sx = 0, sy = 0, sz = 0, cnt = 0;
    for (int zc = 0; zc < nz; zc += kZChunk) {
        const int nzc = min(kZChunk, nz - zc);
        for (int i = threadIdx.x; i < nzc; i += blockDim.x) {
            zy[0][i] = zy[2][i] = INT_MAX;
            zy[1][i] = zy[3][i] = -1;
        }
        __syncthreads();
        const int wend = (zc + nzc) * slice_w;
        for (int w = zc * slice_w + threadIdx.x; w < wend; w += blockDim.x) {
            const uint32_t a = P0[w], b = P1[w];
            if (a | b) {
                const int row = w / nxw;
                const int wx = w - row * nxw;
                const int z = row / ny, y = row - z * ny;
                bx[0] = min(bx[0], z);
                bx[1] = max(bx[1], z);
                bx[2] = min(bx[2], y);
                bx[3] = max(bx[3], y);
                if (a) {
                    atomicMin(&zy[0][z - zc], y);
                    atomicMax(&zy[1][z - zc], y);
                }
                if (b) {
                    bx[4] = min(bx[4], z);
                    bx[5] = max(bx[5], z);
                    bx[6] = min(bx[6], y);
                    bx[7] = max(bx[7], y);
                    atomicMin(&zy[2][z - zc], y);
                    atomicMax(&zy[3][z - zc], y);
                }
                const uint32_t c = popc(a);
                cnt += c;
                sx += (uint64_t)(32u * (uint32_t)wx) * c + bit_position_sum(a);
                sy += (uint64_t)y * c;
                sz += (uint64_t)z * c;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nzc; i += blockDim.x) {
            uint32_t *o = zrange + (e * nz + zc + i) * 2;
#pragma unroll
            for (int p = 0; p < 2; ++p)
                o[p] = zy[2 * p + 1][i] < 0 ? 0u
                                            : (uint32_t)zy[2 * p][i] | ((uint32_t)(zy[2 * p + 1][i] + 1) << 16);
        }
        __syncthreads();                        // the next chunk reuses zy
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) bx[i] = (i & 1) ? wave_max(bx[i]) : wave_min(bx[i]);
    sx = wave_sum64(sx);
    sy = wave_sum64(sy);
    sz = wave_sum64(sz);
    cnt = wave_sum64(cnt);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[wv][i] = bx[i];
        rm[wv][0] = sx;
        rm[wv][1] = sy;
        rm[wv][2] = sz;
        rm[wv][3] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 1; i < nw; ++i) {
#pragma unroll
            for (int t = 0; t < 8; ++t) bx[t] = (t & 1) ? max(bx[t], rb[i][t]) : min(bx[t], rb[i][t]);
            sx += rm[i][0];
            sy += rm[i][1];
            sz += rm[i][2];
            cnt += rm[i][3];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int32_t *b = (h ? tbox : box) + 4 * e;
            const int *x = bx + 4 * h;
            if (x[1] < 0) {
                b[0] = b[1] = b[2] = b[3] = 0;   // no set bit: an empty box
            } else {
                b[0] = x[0];
                b[1] = x[1] + 1;
                b[2] = x[2];
                b[3] = x[3] + 1;
            }
        }
        uint64_t *m = mom + 4 * e;
        m[0] = sx;
        m[1] = sy;
        m[2] = sz;
        m[3] = cnt;
    }
}

hipError_t launch_meta(const uint32_t *recs, int64_t n, const Geometry &g, int32_t *box,
                       int32_t *tbox, uint64_t *mom, uint32_t *zrange, hipStream_t s)
{
    hipLaunchKernelGGL(meta_kernel, dim3((unsigned)n), dim3(256), 0, s, recs, 2 * (int64_t)g.Wp,
                       g.Wp, g.W, g.nxw, g.ny, box, tbox, mom, zrange);
    return hipGetLastError();
}

// z-offset of flattened row r of a box nyr rows wide: r / nyr through a float
// reciprocal (r < 2^24, so the estimate is off by at most one) and a fix-up.
__device__ __forceinline__ int row_div(int r, int nyr, float inv)
{
    int zr = (int)((float)r * inv);
    if (zr * nyr > r) --zr;
    else if ((zr + 1) * nyr <= r) ++zr;
    return zr;
}

// One wave per entry, four entries per 256-thread block. Lanes sweep the
// flattened rows of (entry box n query box); x-rows of 128 voxels (nxw == 4)
// are single 16-byte loads, other widths go word by word.
constexpr int kZStageScan = 128;   // z-slices of the entry's row ranges a wave stages in LDS

template <bool V4, int U>
__global__ void __launch_bounds__(256) box_scan_kernel(const uint32_t *__restrict__ planes, int Wp,
                                                       int nxw, int ny, int nz,
                                                       const int32_t *__restrict__ box,
                                                       const int32_t *__restrict__ tbox,
                                                       const uint32_t *__restrict__ zrange,
                                                       const uint32_t *__restrict__ qpack,
                                                       const int32_t *__restrict__ qbox,
                                                       const int32_t *__restrict__ qtbox, int64_t n,
                                                       uint32_t *__restrict__ inter)
{
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= n) return;   // a whole wave leaves; the kernel has no block barrier
    const int32_t *b = box + 4 * e, *tb = tbox + 4 * e;
    const int z0 = max(b[0], qbox[0]), z1 = min(b[1], qbox[1]);
    const int y0 = max(b[2], qbox[2]), y1 = min(b[3], qbox[3]);
    // The T1Gd plane only inside both T1Gd boxes (a part of the box swept: each T1Gd box lies
    // inside its side's box of both masks).
    const int tz0 = max(tb[0], qtbox[0]), tz1 = min(tb[1], qtbox[1]);
    const int ty0 = max(tb[2], qtbox[2]), ty1 = min(tb[3], qtbox[3]);
    const int nyr = y1 - y0;
    const int nr = (z1 > z0 && nyr > 0) ? (z1 - z0) * nyr : 0;
    const float inv = nyr > 0 ? 1.0f / (float)nyr : 0.0f;
    // The entry's per-slice y-ranges of its FLAIR and T1Gd rows over the slices swept, in this
    // wave's part of LDS (a box deeper than kZStageScan slices goes by the boxes alone).
    __shared__ uint2 s_zr[4][kZStageScan];
    const int wv = threadIdx.x >> 6;
    const bool zr_ok = nr > 0 && z1 - z0 <= kZStageScan;
    if (zr_ok) {
        for (int i = lane; i < z1 - z0; i += 64)
            s_zr[wv][i] = *reinterpret_cast<const uint2 *>(zrange + (e * nz + z0 + i) * 2);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    auto in_range = [&](int z, int y, bool t1gd) {
        if (!zr_ok) return true;
        const uint2 rg = s_zr[wv][z - z0];
        const uint32_t v = t1gd ? rg.y : rg.x;
        return y >= (int)(v & 0xffffu) && y < (int)(v >> 16);
    };
    const uint32_t *D0 = planes + e * 2 * (int64_t)Wp, *D1 = D0 + Wp;
    const uint32_t *Q0 = qpack, *Q1 = qpack + Wp;
    uint32_t c0 = 0, c1 = 0;
    if (V4) {
        for (int r0 = 0; r0 < nr; r0 += 64 * U) {
            u32x4 d0[U], d1[U], q0[U], q1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = r0 + u * 64 + lane;
                d0[u] = d1[u] = q0[u] = q1[u] = (u32x4){0u, 0u, 0u, 0u};
                if (r < nr) {
                    const int zr = row_div(r, nyr, inv);
                    const int z = z0 + zr, y = y0 + r - zr * nyr;
                    const int64_t base = ((int64_t)z * ny + y) * 4;
                    if (in_range(z, y, false)) {
                        d0[u] = load_stream(reinterpret_cast<const u32x4 *>(D0 + base));
                        q0[u] = *reinterpret_cast<const u32x4 *>(Q0 + base);
                    }
                    if (z >= tz0 && z < tz1 && y >= ty0 && y < ty1 && in_range(z, y, true)) {
                        d1[u] = load_stream(reinterpret_cast<const u32x4 *>(D1 + base));
                        q1[u] = *reinterpret_cast<const u32x4 *>(Q1 + base);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c0 += popc_and4(q0[u], d0[u]);
                c1 += popc_and4(q1[u], d1[u]);
            }
        }
    } else {
        const int64_t nt = (int64_t)nr * nxw;
        for (int64_t t = lane; t < nt; t += 64) {
            const int r = (int)(t / nxw), w = (int)(t - (int64_t)r * nxw);
            const int zr = row_div(r, nyr, inv);
            const int z = z0 + zr, y = y0 + r - zr * nyr;
            const int64_t base = ((int64_t)z * ny + y) * nxw + w;
            if (in_range(z, y, false)) c0 += popc(Q0[base] & D0[base]);
            if (z >= tz0 && z < tz1 && y >= ty0 && y < ty1 && in_range(z, y, true))
                c1 += popc(Q1[base] & D1[base]);
        }
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    if (lane == 0) {
        inter[2 * e] = c0;
        inter[2 * e + 1] = c1;
    }
}

hipError_t launch_box_scan(const db_t *db, int64_t n, const uint32_t *qpack, const int32_t *qbox,
                           const int32_t *qtbox, uint32_t *inter, hipStream_t s)
{
    const Geometry &g = db->g;
    const int64_t blocks = (n + 3) / 4;
    if (g.nxw == 4)
        hipLaunchKernelGGL((box_scan_kernel<true, 4>), dim3((unsigned)blocks), dim3(256), 0, s,
                           db->planes, g.Wp, g.nxw, g.ny, g.nz, db->box, db->tbox, db->zrange,
                           qpack, qbox, qtbox, n, inter);
    else
        hipLaunchKernelGGL((box_scan_kernel<false, 1>), dim3((unsigned)blocks), dim3(256), 0, s,
                           db->planes, g.Wp, g.nxw, g.ny, g.nz, db->box, db->tbox, db->zrange,
                           qpack, qbox, qtbox, n, inter);
    return hipGetLastError();
}

// Squared distance between the centres of mass of query q and entry n,
// computed in IEEE double (centre = moment / count, differences squared and
// added x, y, z in that order) and rounded once to float: the selection key.
// An entry or query with an empty FLAIR mask has no centre: +inf, so it
// ranks after every entry that has one (ties by index).
__global__ void __launch_bounds__(256) com_dist_kernel(const uint64_t *__restrict__ qmom,
                                                       const uint64_t *__restrict__ mom, int n,
                                                       float *__restrict__ D)
{
    const int q = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t *a = qmom + 4 * q, *b = mom + 4 * (int64_t)i;
    float out = __builtin_inff();
    if (a[3] != 0 && b[3] != 0) {
        const double qa = (double)a[3], nb = (double)b[3];
        const double dx = (double)a[0] / qa - (double)b[0] / nb;
        const double dy = (double)a[1] / qa - (double)b[1] / nb;
        const double dz = (double)a[2] / qa - (double)b[2] / nb;
        const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        out = (float)((xx + yy) + zz);
    }
    D[(int64_t)q * n + i] = out;
}

hipError_t launch_com_dist(int nq, const uint64_t *qmom, const uint64_t *mom, int n, float *D,
                           hipStream_t s)
{
    hipLaunchKernelGGL(com_dist_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nq), dim3(256),
                       0, s, qmom, mom, n, D);
    return hipGetLastError();
}

}  // namespace tdb
