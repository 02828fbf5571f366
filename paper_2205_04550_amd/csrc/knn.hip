// knn.hip — latent distances and the k nearest database latents per query in one pass,
// with no distance matrix in memory.
//
// Paper Sec. 2.3 ("Autoencoders"): the encoded query is compared with every encoded
// database entry by L2 distance and the lowest wins. The distances are the expanded
// squared form of the distance GEMM (embed.hip), computed by the same instructions in
// the same order, so every distance equals the one emb_distances writes, bit for bit.
// Instead of writing them, each block keeps, for each of its 128 query rows, a running
// bound and a short candidate list:
//
//   - A candidate is packed as fkey(d) << 32 | index: the order of packed values is the
//     order (distance ascending, index ascending), and every packed value of a row is
//     distinct.
//   - Before the full pass, the distance kernel runs over a sample (the first 16,384
//     entries) writing only the smallest key of every group of 16 entries; the k-th
//     smallest of those minima bounds each row for the whole database (k groups, hence
//     k entries, lie at or below it). Databases too small for the sample start without a
//     bound and take one from each block's first tile.
//   - Block (query tile, split) walks the database tiles of its split. A row's bound B is
//     a packed value such that at least k entries are <= B. Every distance with packed
//     <= B is appended to the row's list (a per-lane LDS atomic and a store to the
//     workspace); all others have k better entries and can never be among the k nearest.
//   - When a list outgrows its trigger, one wave tightens B: each lane takes the four
//     smallest keys of the entries it holds, B becomes the k-th smallest of those 256 keys
//     (k distinct entries lie at or below it; bisection on the key with ballot counts),
//     and the list keeps only the entries <= B. When ties on one key would keep more than
//     kKnnKeepMax entries, B becomes the exact k-th smallest packed value instead.
//   - A second kernel merges the splits of a row: B* = the smallest bound over its
//     splits is a bound for the whole row, the entries <= B* of all its lists are
//     gathered, and a radix select on the packed values finds the k smallest, which are
//     sorted and written.
// The result is the k smallest (distance, index) of the row — what emb_topk_min gives
// for the written distances.
#include <limits.h>

#include "common.hpp"
#include "embed_core.hpp"
#include "internal.hpp"

namespace tdb {

constexpr int kKnnCap = 1024;                 // list entries per (block, row)
constexpr int kKnnTrigger = kKnnCap - kDN;    // a list holding more is compacted
constexpr int kKnnKeepMax = 512;              // more kept by the key bound: exact bound
constexpr int kKnnFinal = 512;                // a longer list is tightened at the end
constexpr int kKnnMaxK = kKnnMaxKPublic;
constexpr int kKnnMaxSplit = 64;

__device__ __forceinline__ uint64_t lanemask_lt64(int lane)
{
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Number of values <= x among the 4 x 64 held by the wave (every lane active).
__device__ __forceinline__ int wave_count_le(const uint32_t (&v)[4], uint32_t x)
{
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) c += __popcll(__ballot(v[q] <= x));
    return c;
}

// The float whose key is the high half of bound B: every distance whose packed value is
// <= B is <= it (+inf while B has no key yet).
__device__ __forceinline__ float bound_float(uint64_t B)
{
    const uint32_t key = (uint32_t)(B >> 32);
    return key == ~0u ? __int_as_float(0x7f800000) : fkey_inv(key);
}

// The row part of a conservative test on the dot product: with tau the bound's float,
// a distance dv = fl(fl(qn + xn) - 2 dot) <= tau implies dot >= (qn + xn - tau) / 2 - e
// with e below 2^-24 (qn + xn + 2 |tau|) (qn, xn >= 0). The test dot >= alpha + beta, with
// alpha = (qn - tau) / 2 - m (qn + |tau|) and beta = xn / 2 - m xn (m = 4e-7, above six
// units of rounding, which also covers the rounding of alpha + beta), never fails for such
// a distance; distances passing it are tested exactly.
__device__ __forceinline__ float knn_alpha(float qn, float tau)
{
    if (!(tau < __int_as_float(0x7f800000))) return __int_as_float(0xff800000);   // -inf
    return (qn - tau) * 0.5f - 4e-7f * (qn + fabsf(tau));
}

// Tighten the bound of one row and drop the entries above it (one wave, every lane
// active; L is the row's list of n <= kKnnCap entries, *cnt, *bound and *tauf its LDS
// state). The whole list is loaded once, 16 entries per lane.
__device__ __forceinline__ void knn_compact(uint64_t *__restrict__ L, uint32_t *cnt,
                                            uint64_t *bound, float *tauf, float *alpha, float qn,
                                            int k, int lane)
{
    constexpr int R = kKnnCap / 64;
    const int n = (int)*cnt;
    uint64_t B = *bound;
    // Opaque lane index: keeps the compiler from hoisting the 16 entry offsets of the
    // lane out of the kernel's tile loop (they would hold registers for the whole kernel).
    asm volatile("" : "+v"(lane));
    uint64_t e[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = u * 64 + lane;
        e[u] = ~0ull;
        if (u * 64 < n && i < n) e[u] = L[i];
    }
    // The four smallest keys among this lane's entries.
    uint32_t best[4] = {~0u, ~0u, ~0u, ~0u};
#pragma unroll
    for (int u = 0; u < R; ++u) {
        if (u * 64 < n) {                          // uniform: past n the groups are empty
            uint32_t x = (uint32_t)(e[u] >> 32);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = min(best[q], x);
                x = max(best[q], x);
                best[q] = lo;
            }
        }
    }
    // T = the k-th smallest of the 256 (smallest x with at least k values <= x). A value
    // below all ones is a real entry, so k distinct entries have key <= T; T = all ones
    // (too few entries) leaves B as it is. With at most four entries per lane the 256 are
    // all the entries and T is the exact k-th smallest key.
    uint32_t lo = 0, hi = ~0u;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (wave_count_le(best, mid) >= k) hi = mid;
        else lo = mid + 1;
    }
    const uint64_t Bk = ((uint64_t)lo << 32) | 0xffffffffull;
    if (Bk < B) B = Bk;
    const uint64_t lt = lanemask_lt64(lane);
    // Keep the entries <= B, in order (all of them are in registers).
    int kept = 0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const bool keep = u * 64 + lane < n && e[u] <= B;
        const uint64_t m = __ballot(keep);
        if (keep) L[kept + __popcll(m & lt)] = e[u];
        kept += __popcll(m);
    }
    if (kept > kKnnKeepMax) {
        // Many entries share the bound's key: B = the exact k-th smallest packed value.
        uint64_t lo64 = 0, hi64 = B;
        while (lo64 < hi64) {
            const uint64_t mid = lo64 + ((hi64 - lo64) >> 1);
            int c = 0;
#pragma unroll
            for (int u = 0; u < R; ++u) c += __popcll(__ballot(u * 64 + lane < n && e[u] <= mid));
            if (c >= k) hi64 = mid;
            else lo64 = mid + 1;
        }
        B = lo64;
        kept = 0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const bool keep = u * 64 + lane < n && e[u] <= B;
            const uint64_t m = __ballot(keep);
            if (keep) L[kept + __popcll(m & lt)] = e[u];
            kept += __popcll(m);
        }
    }
    if (lane == 0) {
        *cnt = (uint32_t)kept;
        *bound = B;
        *tauf = bound_float(B);
        *alpha = knn_alpha(qn, *tauf);
    }
}

// Block b of G = mt * nsplit: query tile m and split s with b = 8 (m + mt (s / 8)) + s % 8,
// so the blocks of one split (all query tiles) share an XCD and its L2 copy of the split's
// database tiles. Split s takes database tiles [s nt / nsplit, (s + 1) nt / nsplit).
// Outputs per (block, row): the list lists[b][row][0 .. cnt), cnt, and the bound.
// SEEDB: no bound is given; the block's first tile provides one (small databases).
template <bool FP8, bool TAIL, bool SEEDB>
__global__ void __launch_bounds__(kDThreads, 4) knn_kernel(
    int M, int N, int K, int k, int mt, int nsplit, int nt, const uint8_t *__restrict__ Q,
    const float *__restrict__ qs, const float *__restrict__ qn, const uint8_t *__restrict__ X,
    const float *__restrict__ xs, const float *__restrict__ xn, const uint64_t *__restrict__ seed,
    uint64_t *__restrict__ lists, uint32_t *__restrict__ cnt_out, uint64_t *__restrict__ bound_out)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][(kDM + kDN) * kDRow];
    __shared__ __attribute__((aligned(16))) float tv[2][2][kDM + kDN];
    __shared__ uint64_t s_bound[kDM];
    __shared__ uint32_t s_cnt[kDM];
    __shared__ float s_tauf[kDM];
    __shared__ __attribute__((aligned(16))) float s_alpha[kDM];
    __shared__ float s_qn[kDM];
    __shared__ uint32_t s_seed[kDM];
    const int b = blockIdx.x;
    const int m = (b / kXcds) % mt, s = (b / kXcds) / mt * kXcds + b % kXcds;
    const int m0 = m * kDM;
    const int t0 = (int)((int64_t)s * nt / nsplit), t1 = (int)((int64_t)(s + 1) * nt / nsplit);
    const int T = t1 - t0;                                 // database tiles of this block
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *const Lb = lists + (size_t)b * kDM * kKnnCap;
    if (tid < kDM) {
        // A bound given for the whole row (from a sample of the database) holds for every
        // split; without one, the block's first tile provides the first bound. A row past
        // M gets alpha = +inf, so no distance of it passes the test below.
        const uint64_t B = !SEEDB && m0 + tid < M ? seed[m0 + tid] : ~0ull;
        s_bound[tid] = B;
        s_cnt[tid] = 0;
        s_tauf[tid] = bound_float(B);
        s_qn[tid] = qn[min(m0 + tid, M - 1)];
        s_alpha[tid] = m0 + tid < M ? knn_alpha(s_qn[tid], s_tauf[tid]) : __int_as_float(0x7f800000);
        s_seed[tid] = 0;
    }
    const int Kb = FP8 ? K : 2 * K;                        // bytes per row in Q and X
    const int nslices = (2 * K + kDSlice - 1) / kDSlice;   // 32 values per slice
    const int wm = wave >> 2, wn = wave & 3;
    const int half = lane >> 5, r32 = lane & 31;
    const int frow = tid >> 2, fpart = (tid & 3) * 16;
    // 32-bit offsets: the host keeps N Kb (and M Kb) below 4 GiB. The query row is fixed for
    // the block; the two database rows change with the tile being fetched.
    const uint32_t oq = (uint32_t)min(m0 + frow, M - 1) * (uint32_t)Kb;
    uint32_t ox[2] = {0u, 0u};
    u32x4 pre[3];
    float prv[2];
    // Slice sl of the block's tile i into registers (the fetch runs two slices ahead).
    auto fetch = [&](int i, int sl, u32x4 (&dst)[3], float (&dv)[2]) {
        const int n0 = (t0 + i) * kDN;
        if (sl == 0) {
            ox[0] = (uint32_t)min(n0 + frow, N - 1) * (uint32_t)Kb;
            ox[1] = (uint32_t)min(n0 + kDM + frow, N - 1) * (uint32_t)Kb;
        }
        const uint32_t kb = FP8 ? (uint32_t)(sl * (kDSlice / 2) + (fpart >> 1))
                                : (uint32_t)(sl * kDSlice + fpart);
        if (!TAIL || (int)kb < Kb) {
            if (FP8) {
                dst[0] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(Q + oq + kb));
                dst[1] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(X + ox[0] + kb));
                dst[2] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(X + ox[1] + kb));
            } else {
                dst[0] = *reinterpret_cast<const u32x4 *>(Q + oq + kb);
                dst[1] = *reinterpret_cast<const u32x4 *>(X + ox[0] + kb);
                dst[2] = *reinterpret_cast<const u32x4 *>(X + ox[1] + kb);
            }
        } else {
            dst[0] = dst[1] = dst[2] = (u32x4){0u, 0u, 0u, 0u};
        }
        if (sl == 0 && tid < kDM + kDN) {
            if (tid < kDM) {
                const int row = min(m0 + tid, M - 1);
                dv[0] = qn[row];
                if (FP8) dv[1] = qs[row];
            } else {
                const int col = min(n0 + tid - kDM, N - 1);
                dv[0] = xn[col];
                if (FP8) dv[1] = xs[col];
            }
        }
    };
    auto stash = [&](int i, int sl, int buf, const u32x4 (&src)[3], const float (&sv)[2]) {
        uint8_t *Ls = &lds[buf][0];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            *reinterpret_cast<u32x4 *>(&Ls[(j * kDM + frow) * kDRow + fpart]) = src[j];
        if (sl == 0 && tid < kDM + kDN) {
            tv[i & 1][0][tid] = sv[0];
            if (FP8) tv[i & 1][1][tid] = sv[1];
        }
    };
    f32x16 acc[2][2];
    // The first slice of a tile starts its products from zero (not from the accumulators),
    // so the accumulators are free between a tile's epilogue and its successor's first slice.
    auto compute = [&](int buf, bool first) {
        const uint8_t *A = &lds[buf][0], *Bm = &lds[buf][kDM * kDRow];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            bf16x8 a[2], bb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(
                    A + (wm * 64 + i * 32 + r32) * kDRow + st * 32 + half * 16);
                bb[i] = *reinterpret_cast<const bf16x8 *>(
                    Bm + (wn * 64 + i * 32 + r32) * kDRow + st * 32 + half * 16);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (st == 0 && first) {
                        const f32x16 z = {};
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bb[j], z, 0, 0,
                                                                            0);
                    } else {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bb[j],
                                                                            acc[i][j], 0, 0, 0);
                    }
                }
        }
    };
    // The distances of a finished tile (the arithmetic of the distance kernel's epilogue),
    // appended to the lists of their rows where they are within the rows' bounds. The
    // lanes that hold such a distance each reserve a place in the row's list with an LDS
    // atomic; most (row, column) pairs fail a two-operation test first.
    //
    // seed (the block's first tile, when no bound was given): first a bound from the tile
    // itself. The 64 distances a wave holds for one row are split over the 32 lanes of a
    // half-wave (two per lane); each of the 4 waves sharing the row finds the q-th
    // smallest key of its 64 (q = ceil(k / 4); bisection on the key, ballot counts), and
    // the row's bound is the largest of the 4: at least 4 q >= k distinct entries of the
    // tile lie at or below it.
    auto epilogue = [&](int i_tile, bool seedb) {
        const int n0 = (t0 + i_tile) * kDN;
        const float(&t)[2][kDM + kDN] = tv[i_tile & 1];
        // The lane's first row, made opaque here so that the compiler does not hoist the
        // row addresses of the lists out of the tile loop (they would be spilled).
        int rbase = wm * 64 + 4 * half;
        asm volatile("" : "+v"(rbase));
        // Per column of the lane: its index, norm, scale and the column part of the test
        // (+inf past N, so that no distance of it passes).
        uint32_t colv[2];
        float xc[2], scol[2], beta[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int cl = wn * 64 + j * 32 + r32;
            colv[j] = (uint32_t)(n0 + cl);
            xc[j] = t[0][kDM + cl];
            scol[j] = FP8 ? t[1][kDM + cl] : 1.0f;
            beta[j] = n0 + cl < N ? xc[j] * 0.5f - 4e-7f * xc[j] : __int_as_float(0x7f800000);
        }
        auto append = [&](int rl, int j, float dv) {
            const uint64_t p = ((uint64_t)fkey(dv) << 32) | colv[j];
            if (p <= s_bound[rl]) {
                const uint32_t pos = atomicAdd(&s_cnt[rl], 1u);
                // Opaque row: the list address is formed here, on the rare path, not kept
                // live across the epilogue.
                int ro = rl;
                asm volatile("" : "+v"(ro));
                Lb[(uint32_t)ro * (uint32_t)kKnnCap + pos] = p;
            }
        };
        if constexpr (SEEDB) {
            auto dist = [&](int i, int j, int r, int rl) {
                const float dot = FP8 ? (t[1][rl] * scol[j]) * acc[i][j][r] : acc[i][j][r];
                const float dv = (t[0][rl] + xc[j]) - 2.0f * dot;
                // An entry outside the matrix gets NaN: it passes no test below.
                return (m0 + rl < M && (int)colv[j] < N) ? dv : __int_as_float(0x7fc00000);
            };
            // Distances into the accumulators, then (first tile) the bound.
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j][r] = dist(i, j, r, rbase + i * 32 + 8 * (r >> 2) + (r & 3));
            if (seedb) {
                const int q = (k + 3) / 4;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int rl = rbase + i * 32 + 8 * (r >> 2) + (r & 3);
                        uint32_t kj[2];
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const float v = acc[i][j][r];
                            kj[j] = v == v ? fkey(v) : ~0u;
                        }
                        uint32_t lo = 0, hi = ~0u;          // uniform within each half-wave
                        for (int step = 0; step < 32; ++step) {
                            const uint32_t mid = lo + ((hi - lo) >> 1);
                            const uint64_t a = __ballot(kj[0] <= mid), bb = __ballot(kj[1] <= mid);
                            const uint32_t c =
                                half ? __popc((uint32_t)(a >> 32)) + __popc((uint32_t)(bb >> 32))
                                     : __popc((uint32_t)a) + __popc((uint32_t)bb);
                            if (c >= (uint32_t)q) hi = mid;
                            else lo = mid + 1;
                        }
                        if (r32 == 0) atomicMax(&s_seed[rl], lo);
                    }
                __syncthreads();
                if (tid < kDM) {
                    const uint32_t T = s_seed[tid];
                    const uint64_t Bt = T == ~0u ? ~0ull : (((uint64_t)T << 32) | 0xffffffffull);
                    if (Bt < s_bound[tid]) {
                        s_bound[tid] = Bt;
                        s_tauf[tid] = bound_float(Bt);
                        s_alpha[tid] = knn_alpha(s_qn[tid], s_tauf[tid]);
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int rl = rbase + i * 32 + 8 * (r >> 2) + (r & 3);
                    const float tau = s_tauf[rl];
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (acc[i][j][r] <= tau) append(rl, j, acc[i][j][r]);
                }
        } else {
            // The conservative test on the dot product, four rows (consecutive in the
            // accumulator layout) per LDS read of their row terms.
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int rl0 = rbase + i * 32 + 8 * a;
                    const f32x4 al = *reinterpret_cast<const f32x4 *>(&s_alpha[rl0]);
                    f32x4 sr = {1.0f, 1.0f, 1.0f, 1.0f};
                    if (FP8) sr = *reinterpret_cast<const f32x4 *>(&t[1][rl0]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int r = 4 * a + c;
                        float dt[2];
                        bool ok[2];
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            dt[j] = FP8 ? (sr[c] * scol[j]) * acc[i][j][r] : acc[i][j][r];
                            ok[j] = dt[j] >= al[c] + beta[j];
                        }
                        if (ok[0] || ok[1]) {
                            const float qr = t[0][rl0 + c];
#pragma unroll
                            for (int j = 0; j < 2; ++j)
                                if (ok[j]) append(rl0 + c, j, (qr + xc[j]) - 2.0f * dt[j]);
                        }
                    }
                }
        }
    };
    // Slice positions (tile, K slice) of the next slice to stash and to fetch; each step
    // advances them by one slice.
    auto advance = [&](int &i, int &sl) {
        if (++sl == nslices) {
            sl = 0;
            ++i;
        }
    };
    int si = 0, ssl = 0, fi = 0, fsl = 0;
    __syncthreads();
    if (T > 0) {
        fetch(0, 0, pre, prv);
        stash(0, 0, 0, pre, prv);
        advance(si, ssl);
        fi = si;
        fsl = ssl;
        if (fi < T) fetch(fi, fsl, pre, prv);
        advance(fi, fsl);
        __syncthreads();
    }
    // Slice u of the block's stream is multiplied from LDS buffer u % 2 while slice u + 1 is
    // stashed into the other buffer and slice u + 2 is fetched. The first slice of a tile is
    // peeled off the slice loop, so the accumulators are dead between a tile's epilogue and
    // the next tile (the list compaction uses those registers).
    int u = 0;
    auto step = [&](bool first) {
        compute(u & 1, first);
        if (si < T) {
            stash(si, ssl, (u + 1) & 1, pre, prv);
            advance(si, ssl);
            if (fi < T) {
                fetch(fi, fsl, pre, prv);
                advance(fi, fsl);
            }
        }
        ++u;
    };
    for (int tile = 0; tile < T; ++tile) {
        step(true);
        for (int sl = 1; sl < nslices; ++sl) {
            __syncthreads();
            step(false);
        }
        epilogue(tile, tile == 0);
        __syncthreads();                           // every append of the tile is done
        // A list that outgrows the trigger is tightened.
        for (int rl = wave; rl < kDM; rl += kDThreads / 64)
            if (s_cnt[rl] > (uint32_t)kKnnTrigger)
                knn_compact(Lb + (size_t)rl * kKnnCap, &s_cnt[rl], &s_bound[rl], &s_tauf[rl],
                            &s_alpha[rl], s_qn[rl], k, lane);
        __syncthreads();
    }
    // Long lists are tightened once more (fewer entries for the merge); then the results.
    for (int rl = wave; rl < kDM; rl += kDThreads / 64)
        if (s_cnt[rl] > (uint32_t)kKnnFinal)
            knn_compact(Lb + (size_t)rl * kKnnCap, &s_cnt[rl], &s_bound[rl], &s_tauf[rl],
                        &s_alpha[rl], s_qn[rl], k, lane);
    __syncthreads();
    if (tid < kDM) {
        cnt_out[(size_t)b * kDM + tid] = s_cnt[tid];
        bound_out[(size_t)b * kDM + tid] = s_bound[tid];
    }
}

constexpr int kMergeThreads = 256;
constexpr int kDirectPairs = 4;      // (query, candidate) pairs per wave of knn_direct_kernel
constexpr int kMergeCap = 8192;     // gathered candidates held in LDS

// One block per query row: the k smallest packed values over the row's split lists.
__global__ void __launch_bounds__(kMergeThreads) knn_merge_kernel(
    int k, int mt, int nsplit, const uint64_t *__restrict__ lists,
    const uint32_t *__restrict__ cnt, const uint64_t *__restrict__ bound, int32_t *__restrict__ idx,
    float *__restrict__ dout)
{
    __shared__ uint64_t buf[kMergeCap];
    __shared__ uint64_t win[kKnnMaxK];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_blk[kKnnMaxSplit], s_n[kKnnMaxSplit], s_off[kKnnMaxSplit + 1];
    __shared__ uint64_t s_B;
    __shared__ uint32_t s_gather, s_win, s_sel[3];
    __shared__ unsigned long long s_lo, s_hi;
    const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int m = q / kDM, r = q % kDM;
    // The first wave: lane s reads split s's list length and bound; B* is their smallest bound
    // and the lists are laid end to end at the exclusive prefix sums of the lengths.
    if (tid < 64) {
        const int s = tid;
        uint32_t n_s = 0;
        uint64_t B = ~0ull;
        if (s < nsplit) {
            const uint32_t blk = (uint32_t)(kXcds * (m + mt * (s / kXcds)) + s % kXcds);
            s_blk[s] = blk;
            n_s = cnt[(size_t)blk * kDM + r];
            B = bound[(size_t)blk * kDM + r];
        }
        uint32_t incl = n_s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
            const uint64_t b2 = __shfl_xor(B, o, 64);
            B = b2 < B ? b2 : B;
        }
        if (s < nsplit) {
            s_n[s] = n_s;
            s_off[s] = incl - n_s;
        }
        if (s == nsplit - 1) s_off[nsplit] = incl;
        if (s == 0) {
            s_B = B;
            s_gather = 0;
            s_win = 0;
            s_lo = ~0ull;
            s_hi = 0;
        }
    }
    __syncthreads();
    const uint64_t Bs = s_B;
    const uint32_t n_all = s_off[nsplit];
    // Entry f of the row's lists laid end to end (split by binary search on the offsets).
    auto entry = [&](uint32_t f) {
        int lo = 0, hi = nsplit - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= f) lo = mid;
            else hi = mid - 1;
        }
        return lists[((size_t)s_blk[lo] * kDM + r) * kKnnCap + (f - s_off[lo])];
    };
    // Gather the entries <= B* into LDS while they fit; four loads in flight per thread.
    // Their smallest and largest values fix the bits all of them share. A thread's entries
    // only move forward through the lists, so it keeps the split of its last one.
    uint64_t lo_t = ~0ull, hi_t = 0;
    int sp = 0;
    for (uint32_t f0 = 0; f0 < n_all; f0 += 4 * kMergeThreads) {
        uint64_t e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t f = f0 + u * kMergeThreads + tid;
            e[u] = ~0ull;
            if (f < n_all) {
                while (s_off[sp + 1] <= f) ++sp;      // s_off[nsplit] = n_all > f stops it
                e[u] = lists[((size_t)s_blk[sp] * kDM + r) * kKnnCap + (f - s_off[sp])];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t f = f0 + u * kMergeThreads + tid;
            if (f < n_all && e[u] <= Bs) {
                const uint32_t pos = atomicAdd(&s_gather, 1u);
                if (pos < (uint32_t)kMergeCap) buf[pos] = e[u];
                lo_t = e[u] < lo_t ? e[u] : lo_t;
                hi_t = e[u] > hi_t ? e[u] : hi_t;
            }
        }
    }
    atomicMin(&s_lo, (unsigned long long)lo_t);
    atomicMax(&s_hi, (unsigned long long)hi_t);
    __syncthreads();
    const uint32_t total = s_gather;
    const bool in_lds = total <= (uint32_t)kMergeCap;
    // Radix select on the packed value, 8 bits at a time from the top: after each pass
    // the bin holding the k-th smallest is fixed; once that bin's count equals what is
    // still needed, every candidate whose fixed bits are <= the prefix is a winner.
    const int kk = min(k, (int)min(total, (uint32_t)INT_MAX));
    if (kk == 0) {                          // no candidate (cannot happen for k <= N)
        if (tid < k) {
            idx[(size_t)q * k + tid] = -1;
            dout[(size_t)q * k + tid] = __int_as_float(0x7fc00000);
        }
        return;
    }
    if (tid == 0) s_sel[0] = s_sel[1] = s_sel[2] = 0;
    // The radix passes start at the highest byte in which the candidates differ.
    const uint64_t diff = (uint64_t)s_lo ^ (uint64_t)s_hi;
    const int top = diff ? 63 - __clzll(diff) : 0;
    const int pass0 = 7 - top / 8;
    uint64_t mask = pass0 ? ~0ull << (64 - 8 * pass0) : 0ull;
    uint64_t prefix = (uint64_t)s_lo & mask;
    uint32_t remaining = (uint32_t)kk;
    for (int pass = pass0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        for (int i = tid; i < 256; i += kMergeThreads) hist[i] = 0;
        __syncthreads();
        if (in_lds) {
            for (uint32_t i0 = 0; i0 < total; i0 += kMergeThreads) {
                const uint32_t i = i0 + tid;
                const uint64_t e = i < total ? buf[i] : ~0ull;
                const bool pend = i < total && (e & mask) == prefix;
                hist_add(hist, pend, (uint32_t)(e >> shift) & 255u, lane);
            }
        } else {
            for (uint32_t f0 = 0; f0 < n_all; f0 += kMergeThreads) {
                const uint32_t f = f0 + tid;
                const uint64_t e = f < n_all ? entry(f) : ~0ull;
                const bool pend = f < n_all && e <= Bs && (e & mask) == prefix;
                hist_add(hist, pend, (uint32_t)(e >> shift) & 255u, lane);
            }
        }
        __syncthreads();
        // Inclusive prefix sums of the 256 bins (one wave, four bins per lane).
        if (tid < 64) {
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = hist[4 * tid + u];
                sum += c[u];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t ex = run;
                run += c[u];
                if (ex < remaining && run >= remaining) {
                    s_sel[0] = (uint32_t)(4 * tid + u);
                    s_sel[1] = remaining - ex;      // still needed from this bin
                    s_sel[2] = c[u];                // in this bin
                }
            }
        }
        __syncthreads();
        prefix |= (uint64_t)s_sel[0] << shift;
        mask |= (uint64_t)255 << shift;
        remaining = s_sel[1];
        const bool done = s_sel[1] == s_sel[2];
        __syncthreads();
        if (done) break;
    }
    // Winners: every candidate whose fixed bits are <= the prefix (exactly kk of them).
    auto take = [&](uint64_t e, bool ok) {
        if (ok && (e & mask) <= prefix) {
            const uint32_t pos = atomicAdd(&s_win, 1u);
            if (pos < (uint32_t)kKnnMaxK) win[pos] = e;
        }
    };
    if (in_lds) {
        for (uint32_t i = tid; i < total; i += kMergeThreads) take(buf[i], true);
    } else {
        for (uint32_t f = tid; f < n_all; f += kMergeThreads) {
            const uint64_t e = entry(f);
            take(e, e <= Bs);
        }
    }
    __syncthreads();
    // Sort the winners (padded to 256) ascending in one wave: four per lane, element
    // e = 64 u + lane, bitonic network (partners across lanes by shuffle, across
    // registers in place); no block barrier.
    if (tid >= 64) return;
    uint64_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = 64 * u + lane < kk ? win[64 * u + lane] : ~0ull;
    auto shfl64 = [&](uint64_t x, int src) {
        const uint32_t lo = __shfl((uint32_t)x, src, 64), hi = __shfl((uint32_t)(x >> 32), src, 64);
        return ((uint64_t)hi << 32) | lo;
    };
#pragma unroll
    for (int size = 2; size <= kKnnMaxK; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = 64 * u + lane;
                const bool up = (e & size) == 0, lower = (e & stride) == 0;
                uint64_t o;
                if (stride >= 64) {
                    const int pu = u ^ (stride >> 6);
                    if (pu < u) continue;               // the pair is handled once, from below
                    o = w[pu];
                    const uint64_t mn = o < w[u] ? o : w[u], mx = o < w[u] ? w[u] : o;
                    w[u] = up ? mn : mx;
                    w[pu] = up ? mx : mn;
                    continue;
                }
                o = shfl64(w[u], lane ^ stride);
                w[u] = (lower == up) ? (o < w[u] ? o : w[u]) : (o > w[u] ? o : w[u]);
            }
        }
    uint64_t v = w[0];
    (void)v;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = 64 * u + lane;
        if (e < k) {
            idx[(size_t)q * k + e] = e < kk ? (int32_t)(uint32_t)w[u] : -1;
            dout[(size_t)q * k + e] = e < kk ? fkey_inv((uint32_t)(w[u] >> 32)) : __int_as_float(0x7fc00000);
        }
    }
}

// Direct-form squared distances of given pairs: d = sum_i (q_i - x_i)^2 over the stored
// (dequantised) values, summed in double and rounded once to float; exactly 0 for equal
// codes and scales. A wave takes kDirectPairs pairs (their loads all in flight together),
// four waves per block; each pair's terms are summed in the same order as one pair alone.
template <bool FP8>
__global__ void __launch_bounds__(256) knn_direct_kernel(int M, int N, int k, int K,
                                                         const uint8_t *__restrict__ Q,
                                                         const float *__restrict__ qs,
                                                         const uint8_t *__restrict__ X,
                                                         const float *__restrict__ xs,
                                                         const int32_t *__restrict__ idx,
                                                         float *__restrict__ d)
{
    constexpr int P = kDirectPairs;
    const int lane = threadIdx.x & 63;
    const int64_t pair0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * P;
    const int64_t npairs = (int64_t)M * k;
    if (pair0 >= npairs) return;                  // whole wave
    // The wave's P pairs: their candidates first, then every row they need, all in flight.
    int q[P];
    int32_t e[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int64_t pair = pair0 + j;
        q[j] = pair < npairs ? (int)(pair / k) : 0;
        e[j] = pair < npairs ? idx[pair] : -1;
    }
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    // Eight values per lane per step (K % 8 == 0; rows 8-byte (FP8) / 16-byte (BF16) aligned).
    for (int i0 = lane * 8; i0 < K; i0 += 512) {
        u32x4 a[P], c[P];
        double sa[P], sc[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const bool live = e[j] >= 0 && e[j] < N;
            const int ej = live ? e[j] : 0;
            sa[j] = sc[j] = 1.0;
            if (FP8) {
                a[j] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(Q + (int64_t)q[j] * K + i0));
                c[j] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(X + (int64_t)ej * K + i0));
                sa[j] = qs[q[j]];
                sc[j] = xs[ej];
            } else {
                a[j] = *reinterpret_cast<const u32x4 *>(Q + ((int64_t)q[j] * K + i0) * 2);
                c[j] = *reinterpret_cast<const u32x4 *>(X + ((int64_t)ej * K + i0) * 2);
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int w = 0; w < 4; ++w)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double va = sa[j] * (double)bf16_val((uint16_t)(a[j][w] >> (16 * h)));
                    const double vc = sc[j] * (double)bf16_val((uint16_t)(c[j][w] >> (16 * h)));
                    acc[j] += (va - vc) * (va - vc);
                }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] += __shfl_xor(acc[j], o, 64);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (pair0 + j < npairs && e[j] >= 0 && e[j] < N) d[pair0 + j] = (float)acc[j];
}

// ---- launchers ----

int knn_splits(int M, int N)
{
    (void)M;
    const int nt = (N + kDN - 1) / kDN;
    const int ns = kXcds * (nt / (3 * kXcds));   // at least three tiles per split
    return max(kXcds, min(kKnnMaxSplit, ns));
}

// The row bounds before the full pass. The distance kernel leaves, for the first S
// database entries, the smallest key of every group of 16 consecutive entries; at least
// k groups have a minimum <= the k-th smallest of those minima, so at least k entries of
// the row have a packed value <= (that key, all ones): a bound for the whole row. One
// wave per row; ng <= kSeedMaxGroups groups; no bound (all ones) when ng < k.
constexpr int kSeedMaxGroups = 2048;

__global__ void __launch_bounds__(256) knn_seed_kernel(int M, int ng, int k,
                                                       const uint32_t *__restrict__ gmin,
                                                       uint64_t *__restrict__ seed)
{
    constexpr int R = kSeedMaxGroups / 64;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= M) return;                         // whole wave
    if (ng < k) {
        if (lane == 0) seed[row] = ~0ull;
        return;
    }
    uint32_t v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int g = u * 64 + lane;
        v[u] = g < ng ? gmin[(size_t)row * ng + g] : ~0u;
    }
    // The smallest key with at least k minima <= it (bisection; ballot counts).
    uint32_t lo = 0, hi = ~0u;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        int c = 0;
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (u * 64 < ng) c += __popcll(__ballot(v[u] <= mid));
        if (c >= k) hi = mid;
        else lo = mid + 1;
    }
    if (lane == 0) seed[row] = lo == ~0u ? ~0ull : (((uint64_t)lo << 32) | 0xffffffffull);
}

// Database entries of the sample that bounds every row before the full pass (0: none;
// the blocks then bound their rows from their own first tile).
static int knn_sample_cols(int N)
{
    constexpr int kSample = 16384;
    static_assert(kSample / 16 <= kSeedMaxGroups && kSample / 16 >= kKnnMaxK, "sample size");
    return N >= 2 * kSample ? kSample : 0;
}

size_t knn_ws_bytes(int M, int N)
{
    const size_t G = (size_t)((M + kDM - 1) / kDM) * knn_splits(M, N);
    const size_t S = (size_t)knn_sample_cols(N);
    return align_up(G * kDM * kKnnCap * 8, kAlign) + align_up(G * kDM * 4, kAlign) +
           align_up(G * kDM * 8, kAlign) + align_up((size_t)M * 8, kAlign) +
           align_up((size_t)M * (S / 16) * 4, kAlign);
}

template <bool FP8, bool TAIL, bool SEEDB>
static hipError_t knn_pass(int M, int N, int K, int k, int nsplit, const uint8_t *q, const float *qs,
                           const float *qn, const uint8_t *x, const float *xs, const float *xn,
                           const uint64_t *seed, uint64_t *lists, uint32_t *cnt, uint64_t *bound,
                           hipStream_t s)
{
    const int mt = (M + kDM - 1) / kDM, nt = (N + kDN - 1) / kDN;
    hipLaunchKernelGGL((knn_kernel<FP8, TAIL, SEEDB>), dim3((unsigned)(mt * nsplit)), dim3(kDThreads), 0, s,
                       M, N, K, k, mt, nsplit, nt, q, qs, qn, x, xs, xn, seed, lists, cnt, bound);
    return hipGetLastError();
}

hipError_t launch_knn(bool fp8, int M, int N, int K, const void *Q, const float *qs,
                      const float *qn, const void *X, const float *xs, const float *xn, int k,
                      bool direct, int32_t *idx, float *d, void *ws, hipStream_t s)
{
    const int mt = (M + kDM - 1) / kDM, nsplit = knn_splits(M, N);
    const size_t G = (size_t)mt * nsplit;
    uint64_t *lists = static_cast<uint64_t *>(ws);
    char *p = static_cast<char *>(ws) + align_up(G * kDM * kKnnCap * 8, kAlign);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(p);
    p += align_up(G * kDM * 4, kAlign);
    uint64_t *bound = reinterpret_cast<uint64_t *>(p);
    p += align_up(G * kDM * 8, kAlign);
    uint64_t *seed = reinterpret_cast<uint64_t *>(p);
    p += align_up((size_t)M * 8, kAlign);
    uint32_t *gmin = reinterpret_cast<uint32_t *>(p);
    const auto *q = static_cast<const uint8_t *>(Q);
    const auto *x = static_cast<const uint8_t *>(X);
    const bool tail = !fp8 && (2 * K) % kDSlice;
    hipError_t e = hipSuccess;
    const int S = knn_sample_cols(N);
    if (S) {
        // Group minima of the first S entries (no distances written), then the seeds.
        if (fp8)
            e = launch_dist_fp8(M, S, K, q, qs, qn, x, xs, xn, nullptr, 0, gmin, s);
        else
            e = launch_dist_bf16(M, S, K, static_cast<const uint16_t *>(Q), qn,
                                 static_cast<const uint16_t *>(X), xn, nullptr, 0, gmin, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(knn_seed_kernel, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, M,
                           S / 16, k, gmin, seed);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (fp8)
            e = knn_pass<true, false, false>(M, N, K, k, nsplit, q, qs, qn, x, xs, xn, seed,
                                             lists, cnt, bound, s);
        else if (tail)
            e = knn_pass<false, true, false>(M, N, K, k, nsplit, q, nullptr, qn, x, nullptr, xn,
                                             seed, lists, cnt, bound, s);
        else
            e = knn_pass<false, false, false>(M, N, K, k, nsplit, q, nullptr, qn, x, nullptr, xn,
                                              seed, lists, cnt, bound, s);
    } else {
        if (fp8)
            e = knn_pass<true, false, true>(M, N, K, k, nsplit, q, qs, qn, x, xs, xn, nullptr,
                                            lists, cnt, bound, s);
        else if (tail)
            e = knn_pass<false, true, true>(M, N, K, k, nsplit, q, nullptr, qn, x, nullptr, xn,
                                            nullptr, lists, cnt, bound, s);
        else
            e = knn_pass<false, false, true>(M, N, K, k, nsplit, q, nullptr, qn, x, nullptr, xn,
                                             nullptr, lists, cnt, bound, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)M), dim3(kMergeThreads), 0, s, k, mt,
                       nsplit, lists, cnt, bound, idx, d);
    e = hipGetLastError();
    if (e != hipSuccess || !direct) return e;
    const int64_t pairs = (int64_t)M * k;
    const unsigned dblocks = (unsigned)((pairs + 4 * kDirectPairs - 1) / (4 * kDirectPairs));
    if (fp8)
        hipLaunchKernelGGL((knn_direct_kernel<true>), dim3(dblocks), dim3(256), 0, s, M, N, k, K,
                           q, qs, x, xs, idx, d);
    else
        hipLaunchKernelGGL((knn_direct_kernel<false>), dim3(dblocks), dim3(256), 0, s, M, N, k, K,
                           q, nullptr, x, nullptr, idx, d);
    return hipGetLastError();
}

}  // namespace tdb
