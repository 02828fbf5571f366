// pack.hip — threshold + bit-pack of simulated densities, and packing of query labels.
//
// Paper Sec. 2.3 ("Query to a database of synthetic tumors"): the raw
// simulations are densities in [0, 1]; FLAIR and T1Gd segmentations are
// extracted by thresholding at a lower and a higher level. Here each mask is
// stored as one bit per voxel (LSB-first in uint32 words, x fastest), which
// is all a Dice overlap needs and is 32x smaller than float32.
#include <limits.h>

#include "common.hpp"
#include "internal.hpp"

namespace tdb {

// One block per simulation. Lanes read consecutive 16-byte groups (4 voxels),
// so every load instruction is fully coalesced; the 4-bit nibbles of 8
// neighbouring lanes are OR-ed into one 32-voxel word with three xor shuffles.
// Also counts the mask populations |B_FLAIR|, |B_T1Gd| used by every later Dice.
__global__ void __launch_bounds__(256) pack_db_kernel(const float *__restrict__ conc, int64_t V,
                                                      int W, int Wp, float t_lo, float t_hi,
                                                      uint32_t *__restrict__ planes,
                                                      uint32_t *__restrict__ popcnt)
{
    __shared__ uint32_t red[2 * 4];
    const int64_t s = blockIdx.x;
    const f32x4 *c = reinterpret_cast<const f32x4 *>(conc + s * V);
    uint32_t *o = planes + s * 2 * (int64_t)Wp;
    const int nvec = 8 * W, nall = 8 * Wp;   // 16-byte groups with data / incl. padding words
    const int j = threadIdx.x & 7;
    uint32_t n0 = 0, n1 = 0;
    for (int base = 0; base < nall; base += blockDim.x) {   // uniform trip count
        const int i = base + threadIdx.x;
        uint32_t b0 = 0, b1 = 0;
        if (i < nvec) {
            const f32x4 v = __builtin_nontemporal_load(c + i);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                b0 |= (uint32_t)(v[e] >= t_lo) << e;
                b1 |= (uint32_t)(v[e] >= t_hi) << e;
            }
        }
        b0 <<= 4 * j;
        b1 <<= 4 * j;
#pragma unroll
        for (int o2 = 1; o2 < 8; o2 <<= 1) {
            b0 |= __shfl_xor(b0, o2, 64);
            b1 |= __shfl_xor(b1, o2, 64);
        }
        if (j == 0 && i < nall) {
            const int w = i >> 3;
            o[w] = b0;
            o[Wp + w] = b1;
            n0 += popc(b0);
            n1 += popc(b1);
        }
    }
    block_sum2(n0, n1, red);
    if (threadIdx.x == 0) {
        popcnt[2 * s] = n0;
        popcnt[2 * s + 1] = n1;
    }
}

hipError_t launch_pack_db(const db_t *db, const float *conc, int64_t n, uint32_t *planes,
                          uint32_t *popcnt, hipStream_t s)
{
    const Geometry &g = db->g;
    // One launch per at most 2^31-1 simulations is far beyond any capacity.
    hipLaunchKernelGGL(pack_db_kernel, dim3((unsigned)n), dim3(256), 0, s, conc, g.V, g.W, g.Wp,
                       db->t_lo, db->t_hi, planes, popcnt);
    return hipGetLastError();
}

// Bits of word w of one mask that lie inside the ROI (all ones without ROI).
__device__ __forceinline__ uint32_t roi_word_mask(const int32_t *r, int w, int nxw, int ny)
{
    const int wx = w % nxw;
    const int row = w / nxw;
    const int y = row % ny;
    const int z = row / ny;
    if (z < r[2] || z >= r[5] || y < r[1] || y >= r[4])
        return 0u;
    const int lo = r[0] - 32 * wx;  // first voxel of the box relative to the word
    const int hi = r[3] - 32 * wx;  // one past the last
    if (hi <= 0 || lo >= 32)
        return 0u;
    uint32_t m = 0xffffffffu;
    if (lo > 0) m &= 0xffffffffu << lo;
    if (hi < 32) m &= (1u << hi) - 1u;
    return m;
}

constexpr int kPackBatch = 8;


// A block's share of a query's statistics: mask counts, the row range of set bits
// and the FLAIR moments (sum of x, y, z over its bits), summed over packed words.
struct PartAcc {
    uint32_t n0 = 0, n1 = 0;
    int zlo = INT_MAX, zhi = -1, ylo = INT_MAX, yhi = -1;
    int tzlo = INT_MAX, tzhi = -1, tylo = INT_MAX, tyhi = -1;   // rows with a T1Gd bit
    uint64_t sx = 0, sy = 0, sz = 0;

    __device__ void add_t1gd_row(int z, int y)
    {
        tzlo = min(tzlo, z);
        tzhi = max(tzhi, z);
        tylo = min(tylo, y);
        tyhi = max(tyhi, y);
    }

    __device__ void add(uint32_t b0, uint32_t b1, int w, int nxw, int ny)
    {
        n0 += popc(b0);
        n1 += popc(b1);
        if (b0 | b1) {
            const int row = w / nxw;
            const int wx = w - row * nxw;
            const int z = row / ny, y = row - z * ny;
            zlo = min(zlo, z);
            zhi = max(zhi, z);
            ylo = min(ylo, y);
            yhi = max(yhi, y);
            if (b1) add_t1gd_row(z, y);
            const uint32_t c = popc(b0);
            sx += (uint64_t)(32u * (uint32_t)wx) * c + bit_position_sum(b0);
            sy += (uint64_t)y * c;
            sz += (uint64_t)z * c;
        }
    }

    // Block-wide sum (at most 4 waves); thread 0 writes the part.
    __device__ void write(QueryPart &p)
    {
        __shared__ uint32_t rc[4][2];
        __shared__ int rb[4][8];
        __shared__ uint64_t rm[4][3];
        n0 = wave_sum(n0);
        n1 = wave_sum(n1);
        zlo = wave_min(zlo);
        ylo = wave_min(ylo);
        zhi = wave_max(zhi);
        yhi = wave_max(yhi);
        tzlo = wave_min(tzlo);
        tylo = wave_min(tylo);
        tzhi = wave_max(tzhi);
        tyhi = wave_max(tyhi);
        sx = wave_sum64(sx);
        sy = wave_sum64(sy);
        sz = wave_sum64(sz);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            rc[wv][0] = n0;
            rc[wv][1] = n1;
            rb[wv][0] = zlo;
            rb[wv][1] = zhi;
            rb[wv][2] = ylo;
            rb[wv][3] = yhi;
            rb[wv][4] = tzlo;
            rb[wv][5] = tzhi;
            rb[wv][6] = tylo;
            rb[wv][7] = tyhi;
            rm[wv][0] = sx;
            rm[wv][1] = sy;
            rm[wv][2] = sz;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
                n0 += rc[i][0];
                n1 += rc[i][1];
                zlo = min(zlo, rb[i][0]);
                zhi = max(zhi, rb[i][1]);
                ylo = min(ylo, rb[i][2]);
                yhi = max(yhi, rb[i][3]);
                tzlo = min(tzlo, rb[i][4]);
                tzhi = max(tzhi, rb[i][5]);
                tylo = min(tylo, rb[i][6]);
                tyhi = max(tyhi, rb[i][7]);
                sx += rm[i][0];
                sy += rm[i][1];
                sz += rm[i][2];
            }
            p.cnt[0] = n0;
            p.cnt[1] = n1;
            p.box[0] = zlo;
            p.box[1] = zhi;
            p.box[2] = ylo;
            p.box[3] = yhi;
            p.tbox[0] = tzlo;
            p.tbox[1] = tzhi;
            p.tbox[2] = tylo;
            p.tbox[3] = tyhi;
            p.mom[0] = sx;
            p.mom[1] = sy;
            p.mom[2] = sz;
        }
    }
};

// grid (kQueryParts, nq): labels uint8 [nq][V] -> packed [nq][2][Wp] and one
// QueryPart per block: the block's mask counts, the row range of its set bits
// and the FLAIR moments (for the row-box scan and the centre-of-mass key).
// With rois, bits outside the box are cleared first, so later overlaps need no
// masking of the query side.
__global__ void __launch_bounds__(256) pack_query_kernel(const uint8_t *__restrict__ labels,
                                                         int64_t V, int W, int Wp, int nxw, int ny,
                                                         const int32_t *__restrict__ rois,
                                                         uint32_t *__restrict__ qpack,
                                                         QueryPart *__restrict__ qpart)
{
    const int q = blockIdx.y;
    const u32x4 *lab = reinterpret_cast<const u32x4 *>(labels + (int64_t)q * V);
    uint32_t *o = qpack + (int64_t)q * 2 * Wp;
    const int32_t *r = rois ? rois + 6 * q : nullptr;
    PartAcc acc;
    // Two lanes per packed word, 16 label bytes each, so one load instruction covers
    // 1 KiB of contiguous labels; each block packs one contiguous run of words,
    // kPackBatch words per lane pair and pass with all their loads issued first. The
    // even lane assembles the word from both halves.
    const int half = threadIdx.x & 1;
    const int stride = blockDim.x >> 1;
    const int seg = (Wp + gridDim.x - 1) / gridDim.x;
    const int wbeg = blockIdx.x * seg, wend = min(Wp, wbeg + seg);
    for (int w0 = wbeg + (threadIdx.x >> 1); w0 - (int)(threadIdx.x >> 1) < wend;
         w0 += kPackBatch * stride) {
        u32x4 vb[kPackBatch];
#pragma unroll
        for (int u = 0; u < kPackBatch; ++u) {
            const int w = w0 + u * stride;
            vb[u] = (u32x4){0u, 0u, 0u, 0u};
            if (w < W && w < wend) vb[u] = load_stream(lab + 2 * (int64_t)w + half);
        }
#pragma unroll
        for (int u = 0; u < kPackBatch; ++u) {
            const int w = w0 + u * stride;
            uint32_t h0 = 0, h1 = 0;   // this lane's 16 bits of each mask
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t f4, t4;
                label_nibbles(vb[u][e], f4, t4);
                h0 |= f4 << (4 * e);
                h1 |= t4 << (4 * e);
            }
            const uint32_t g0 = __shfl_down(h0, 1, 64), g1 = __shfl_down(h1, 1, 64);
            if (half || w >= wend) continue;
            uint32_t b0 = h0 | (g0 << 16), b1 = h1 | (g1 << 16);
            if (w < W && r) {
                const uint32_t m = roi_word_mask(r, w, nxw, ny);
                b0 &= m;
                b1 &= m;
            }
            if (w < W) acc.add(b0, b1, w, nxw, ny);
            o[w] = b0;
            o[Wp + w] = b1;
        }
    }
    acc.write(qpart[(int64_t)q * kQueryParts + blockIdx.x]);
}

hipError_t launch_pack_queries(const db_t *db, const uint8_t *labels, int nq, const int32_t *rois,
                               uint32_t *qpack, QueryPart *qpart, hipStream_t s)
{
    const Geometry &g = db->g;
    hipLaunchKernelGGL(pack_query_kernel, dim3(kQueryParts, nq), dim3(256), 0, s, labels, g.V,
                       g.W, g.Wp, g.nxw, g.ny, rois, qpack, qpart);
    return hipGetLastError();
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr int kPoolBatch = 2;   // lane units per pass of pack_pool_query_kernel, loads first

// Swap the bits of x selected by mask with the bits d places above them.
__device__ __forceinline__ uint32_t delta_swap(uint32_t x, uint32_t mask, int d)
{
    const uint32_t t = ((x >> d) ^ x) & mask;
    return x ^ t ^ (t << d);
}

// The two mask bits of 16 label bytes (x[q] byte r = voxel 4 q + r) as one word: FLAIR of
// voxel k at bit k, T1Gd of voxel k at bit 16 + k. The masked words are merged so that
// bit 8 r + 2 q + p holds mask p of voxel 4 q + r; four swaps of index bits (r1 with p, then
// r0 past q1 and q0 to the bottom) put it at 16 p + 4 q + r.
__device__ __forceinline__ uint32_t gather_masks(const uint32_t (&a)[4])
{
    uint32_t z = a[0] | (a[1] << 2) | (a[2] << 4) | (a[3] << 6);
    z = delta_swap(z, 0x0000aaaau, 15);
    z = delta_swap(z, 0x00f000f0u, 4);
    z = delta_swap(z, 0x0c0c0c0cu, 2);
    return delta_swap(z, 0x22222222u, 1);
}

// grid (kQueryParts, nq): pack_query_kernel's outputs (no ROI) and, from the same read of
// the labels, their pooled counts for the encoder's first layer: uint8 [nq][nz/2][ny/2][nx/2],
// per 2x2x2 block of voxels its FLAIR count (0..8) in bits 0..3 and its T1Gd count in bits
// 4..7. Needs ny and nz even. A lane unit is 16 voxels along x in each of the four rows
// (2 pz + dz, 2 py + dy), 16 label bytes per row; the two units of one word form a lane pair:
// per row the even lane stores the FLAIR word and the odd lane the T1Gd word (one exchange),
// and each lane sums its bytes into the 8 pooled counts of its 16 voxels.
__global__ void __launch_bounds__(256) pack_pool_query_kernel(const uint8_t *__restrict__ labels,
                                                              int64_t V, int Wp, int nx,
                                                              int ny, uint32_t *__restrict__ qpack,
                                                              QueryPart *__restrict__ qpart,
                                                              uint8_t *__restrict__ pooled)
{
    const int q = blockIdx.y;
    const u32x4 *lab = reinterpret_cast<const u32x4 *>(labels + (int64_t)q * V);
    const int half = threadIdx.x & 1;
    uint32_t *o = qpack + (int64_t)q * 2 * Wp + half * Wp;   // this lane's plane
    uint8_t *P = pooled + (int64_t)q * (V >> 3);
    const int nxw = nx >> 5, PY = ny >> 1, PX = nx >> 1, rowv = nx >> 4;   // rowv: u32x4 per row
    // Exchange selector: the even lane keeps its FLAIR half and takes its partner's; the odd
    // lane takes its partner's T1Gd half and keeps its own.
    const uint32_t sel = half ? 0x03020706u : 0x05040100u;
    PartAcc acc;   // with ny, nz even W = nxw ny nz is a multiple of 4: no padding words
    const int U = (int)(V >> 6);                       // lane units; ubeg and seg even
    const int seg = 2 * ((U / 2 + gridDim.x - 1) / gridDim.x);
    const int ubeg = blockIdx.x * seg, uend = min(U, ubeg + seg);
    for (int u0 = ubeg + threadIdx.x; u0 - (int)threadIdx.x < uend;
         u0 += kPoolBatch * blockDim.x) {
        u32x4 v[kPoolBatch][4];
        int xw[kPoolBatch], py[kPoolBatch], pz[kPoolBatch];
#pragma unroll
        for (int i = 0; i < kPoolBatch; ++i) {
            const int u = u0 + i * blockDim.x, pair = u >> 1;
            xw[i] = pair % nxw;
            py[i] = (pair / nxw) % PY;
            pz[i] = pair / (nxw * PY);
            const int64_t row0 = (int64_t)(2 * pz[i]) * ny + 2 * py[i];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[i][r] = (u32x4){0u, 0u, 0u, 0u};
                if (u < uend)
                    v[i][r] = load_stream(lab + (row0 + (r >> 1) * ny + (r & 1)) * rowv +
                                          2 * xw[i] + half);
            }
        }
#pragma unroll
        for (int i = 0; i < kPoolBatch; ++i) {
            const bool valid = u0 + i * (int)blockDim.x < uend;
            // Per byte, over the four rows: S = FLAIR + 2 T1Gd voxels, T2 = 2 T1Gd voxels.
            uint32_t S[4] = {0u, 0u, 0u, 0u}, T2[4] = {0u, 0u, 0u, 0u};
            uint32_t cnt = 0, cdz = 0, cdy = 0, bps = 0;   // this unit's words of this lane's plane
            uint32_t *ow = o + (int64_t)(2 * pz[i] * ny + 2 * py[i]) * nxw + xw[i];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint32_t a[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    a[e] = v[i][r][e] & 0x03030303u;
                    S[e] += a[e];
                    T2[e] += a[e] & 0x02020202u;
                }
                const uint32_t z = gather_masks(a);
                const uint32_t other = __builtin_amdgcn_mov_dpp(z, 0xb1, 0xf, 0xf, true);   // lane ^ 1
                const uint32_t word = __builtin_amdgcn_perm(other, z, sel);
                if (valid) {
                    const int dz = r >> 1, dy = r & 1;
                    ow[(dz * ny + dy) * nxw] = word;
                    const uint32_t c = popc(word);
                    cnt += c;
                    cdz += dz ? c : 0u;
                    cdy += dy ? c : 0u;
                    if (word) {
                        const int zz = 2 * pz[i] + dz, yy = 2 * py[i] + dy;
                        acc.zlo = min(acc.zlo, zz);
                        acc.zhi = max(acc.zhi, zz);
                        acc.ylo = min(acc.ylo, yy);
                        acc.yhi = max(acc.yhi, yy);
                        if (half) acc.add_t1gd_row(zz, yy);
                        else bps += bit_position_sum(word);
                    }
                }
            }
            if (half) {
                acc.n1 += cnt;
            } else {
                acc.n0 += cnt;
                acc.sx += (uint64_t)(32u * (uint32_t)xw[i]) * cnt + bps;
                acc.sy += (uint64_t)(2u * (uint32_t)py[i]) * cnt + cdy;
                acc.sz += (uint64_t)(2u * (uint32_t)pz[i]) * cnt + cdz;
            }
            // Byte pairs (x, x + 1) -> pooled counts: FLAIR in bits 0..3, T1Gd in 4..7 of
            // bytes 0 and 2 of c[e] (pooled x 2 e and 2 e + 1 of this lane's 8).
            uint32_t c[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t b = (S[e] - T2[e]) | (T2[e] << 3);
                c[e] = (b & 0x00ff00ffu) + ((b >> 8) & 0x00ff00ffu);
            }
            if (valid) {
                const u32x2 pw = {__builtin_amdgcn_perm(c[1], c[0], 0x06040200u),
                                  __builtin_amdgcn_perm(c[3], c[2], 0x06040200u)};
                *reinterpret_cast<u32x2 *>(P + ((int64_t)pz[i] * PY + py[i]) * PX + 16 * xw[i] +
                                           8 * half) = pw;
            }
        }
    }
    acc.write(qpart[(int64_t)q * kQueryParts + blockIdx.x]);
}

hipError_t launch_pack_pool_queries(const db_t *db, const uint8_t *labels, int nq,
                                    uint32_t *qpack, QueryPart *qpart, uint8_t *pooled,
                                    hipStream_t s)
{
    const Geometry &g = db->g;
    hipLaunchKernelGGL(pack_pool_query_kernel, dim3(kQueryParts, nq), dim3(256), 0, s, labels,
                       g.V, g.Wp, g.nx, g.ny, qpack, qpart, pooled);
    return hipGetLastError();
}

// One wave per query: combine its kQueryParts partials.
// A row box as [z0, z1) x [y0, y1) from the extreme rows (all zero when there is none).
__device__ __forceinline__ void write_box(int32_t *bx, int zlo, int zhi, int ylo, int yhi)
{
    if (zhi < 0) {
        bx[0] = bx[1] = bx[2] = bx[3] = 0;
    } else {
        bx[0] = zlo;
        bx[1] = zhi + 1;
        bx[2] = ylo;
        bx[3] = yhi + 1;
    }
}

__global__ void __launch_bounds__(64) sum_parts_kernel(const QueryPart *__restrict__ qpart,
                                                      uint32_t *__restrict__ acnt,
                                                      int32_t *__restrict__ qbox,
                                                      uint64_t *__restrict__ qmom,
                                                      int32_t *__restrict__ qtbox)
{
    const int q = blockIdx.x;
    uint32_t a = 0, b = 0;
    int zlo = INT_MAX, zhi = -1, ylo = INT_MAX, yhi = -1;
    int tzlo = INT_MAX, tzhi = -1, tylo = INT_MAX, tyhi = -1;
    uint64_t sx = 0, sy = 0, sz = 0;
    for (int i = threadIdx.x; i < kQueryParts; i += 64) {
        const QueryPart &p = qpart[(int64_t)q * kQueryParts + i];
        a += p.cnt[0];
        b += p.cnt[1];
        zlo = min(zlo, p.box[0]);
        zhi = max(zhi, p.box[1]);
        ylo = min(ylo, p.box[2]);
        yhi = max(yhi, p.box[3]);
        tzlo = min(tzlo, p.tbox[0]);
        tzhi = max(tzhi, p.tbox[1]);
        tylo = min(tylo, p.tbox[2]);
        tyhi = max(tyhi, p.tbox[3]);
        sx += p.mom[0];
        sy += p.mom[1];
        sz += p.mom[2];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    zlo = wave_min(zlo);
    ylo = wave_min(ylo);
    zhi = wave_max(zhi);
    yhi = wave_max(yhi);
    tzlo = wave_min(tzlo);
    tylo = wave_min(tylo);
    tzhi = wave_max(tzhi);
    tyhi = wave_max(tyhi);
    sx = wave_sum64(sx);
    sy = wave_sum64(sy);
    sz = wave_sum64(sz);
    if (threadIdx.x == 0) {
        acnt[2 * q] = a;
        acnt[2 * q + 1] = b;
        write_box(qbox + 4 * q, zlo, zhi, ylo, yhi);
        if (qtbox) write_box(qtbox + 4 * q, tzlo, tzhi, tylo, tyhi);
        uint64_t *m = qmom + 4 * q;
        m[0] = sx;
        m[1] = sy;
        m[2] = sz;
        m[3] = a;
    }
}

hipError_t launch_sum_parts(const QueryPart *qpart, int nq, uint32_t *acnt, int32_t *qbox,
                            uint64_t *qmom, hipStream_t s, int32_t *qtbox)
{
    hipLaunchKernelGGL(sum_parts_kernel, dim3(nq), dim3(64), 0, s, qpart, acnt, qbox, qmom,
                       qtbox);
    return hipGetLastError();
}

__global__ void fill_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace tdb
