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
//   - Block (query tile, split) walks the database tiles of its split. A row's bound B is
//     a packed value such that at least k entries of the split seen so far are <= B (or
//     all ones while fewer are known). Every distance with packed <= B is appended to the
//     row's list (an LDS counter and a store to the workspace); all others have k better
//     entries in the same split and can never be among the k nearest.
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

// Tighten the bound of one row and drop the entries above it (one wave, every lane
// active; L is the row's list, *cnt and *bound its LDS state).
__device__ __forceinline__ void knn_compact(uint64_t *__restrict__ L, uint32_t *cnt,
                                                     uint64_t *bound, int k, int lane)
{
    const int n = (int)*cnt;
    uint64_t B = *bound;
    // The four smallest keys among this lane's entries (lane, lane + 64, ...).
    uint32_t best[4] = {~0u, ~0u, ~0u, ~0u};
    for (int j0 = 0; j0 * 64 < n; j0 += 4) {
        uint64_t e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = (j0 + u) * 64 + lane;
            e[u] = i < n ? L[i] : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
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
    // (too few entries) leaves B as it is.
    uint32_t lo = 0, hi = ~0u;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (wave_count_le(best, mid) >= k) hi = mid;
        else lo = mid + 1;
    }
    const uint64_t Bk = ((uint64_t)lo << 32) | 0xffffffffull;
    if (Bk < B) B = Bk;
    const uint64_t lt = lanemask_lt64(lane);
    // Keep the entries <= B in order, in place: a chunk's loads all precede its stores,
    // and stores only reach positions below the chunk's first entry plus its kept count.
    int kept = 0;
    for (int j0 = 0; j0 * 64 < n; j0 += 4) {
        uint64_t e[4];
        bool keep[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = (j0 + u) * 64 + lane;
            e[u] = i < n ? L[i] : ~0ull;
            keep[u] = i < n && e[u] <= B;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t m = __ballot(keep[u]);
            if (keep[u]) L[kept + __popcll(m & lt)] = e[u];
            kept += __popcll(m);
        }
    }
    if (kept > kKnnKeepMax) {
        // Many entries share the bound's key: B = the exact k-th smallest packed value.
        uint64_t lo64 = 0, hi64 = B;
        while (lo64 < hi64) {
            const uint64_t mid = lo64 + ((hi64 - lo64) >> 1);
            int c = 0;
            for (int i0 = 0; i0 < kept; i0 += 64) {
                const int i = i0 + lane;
                c += __popcll(__ballot(i < kept && L[i] <= mid));
            }
            if (c >= k) hi64 = mid;
            else lo64 = mid + 1;
        }
        B = lo64;
        int kk = 0;
        for (int i0 = 0; i0 < kept; i0 += 64) {
            const int i = i0 + lane;
            const uint64_t e = i < kept ? L[i] : ~0ull;
            const bool keep = i < kept && e <= B;
            const uint64_t m = __ballot(keep);
            if (keep) L[kk + __popcll(m & lt)] = e;
            kk += __popcll(m);
        }
        kept = kk;
    }
    if (lane == 0) {
        *cnt = (uint32_t)kept;
        *bound = B;
    }
}

// Block b of G = mt * nsplit: query tile m and split s with b = 8 (m + mt (s / 8)) + s % 8,
// so the blocks of one split (all query tiles) share an XCD and its L2 copy of the split's
// database tiles. Split s takes database tiles [s nt / nsplit, (s + 1) nt / nsplit).
// Outputs per (block, row): the list lists[b][row][0 .. cnt), cnt, and the bound.
template <bool FP8, bool TAIL>
__global__ void __launch_bounds__(kDThreads, 4) knn_kernel(
    int M, int N, int K, int k, int mt, int nsplit, int nt, const uint8_t *__restrict__ Q,
    const float *__restrict__ qs, const float *__restrict__ qn, const uint8_t *__restrict__ X,
    const float *__restrict__ xs, const float *__restrict__ xn, uint64_t *__restrict__ lists,
    uint32_t *__restrict__ cnt_out, uint64_t *__restrict__ bound_out)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][(kDM + kDN) * kDRow];
    __shared__ float tv[2][2][kDM + kDN];
    __shared__ uint64_t s_bound[kDM];
    __shared__ uint32_t s_cnt[kDM];
    const int b = blockIdx.x;
    const int m = (b / kXcds) % mt, s = (b / kXcds) / mt * kXcds + b % kXcds;
    const int m0 = m * kDM;
    const int t0 = (int)((int64_t)s * nt / nsplit), t1 = (int)((int64_t)(s + 1) * nt / nsplit);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *const Lb = lists + (size_t)b * kDM * kKnnCap;
    if (tid < kDM) {
        s_bound[tid] = ~0ull;
        s_cnt[tid] = 0;
    }
    const int Kb = FP8 ? K : 2 * K;                        // bytes per row in Q and X
    const int nslices = (2 * K + kDSlice - 1) / kDSlice;   // 32 values per slice
    const int U = (t1 - t0) * nslices;
    const int wm = wave >> 2, wn = wave & 3;
    const int half = lane >> 5, r32 = lane & 31;
    const int frow = tid >> 2, fpart = (tid & 3) * 16;
    u32x4 pre[3];
    float prv[2];
    auto fetch = [&](int v, u32x4 (&dst)[3], float (&dv)[2]) {
        const int i = v / nslices, sl = v - i * nslices;
        const int n0 = (t0 + i) * kDN;
        const uint32_t kb = FP8 ? (uint32_t)(sl * (kDSlice / 2) + (fpart >> 1))
                                : (uint32_t)(sl * kDSlice + fpart);
        if (!TAIL || (int)kb < Kb) {
            const uint64_t o0 = (uint64_t)min(m0 + frow, M - 1) * (uint64_t)Kb + kb;
            const uint64_t o1 = (uint64_t)min(n0 + frow, N - 1) * (uint64_t)Kb + kb;
            const uint64_t o2 = (uint64_t)min(n0 + kDM + frow, N - 1) * (uint64_t)Kb + kb;
            if (FP8) {
                dst[0] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(Q + o0));
                dst[1] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(X + o1));
                dst[2] = e4m3x8_to_bf16(*reinterpret_cast<const u32x2 *>(X + o2));
            } else {
                dst[0] = *reinterpret_cast<const u32x4 *>(Q + o0);
                dst[1] = *reinterpret_cast<const u32x4 *>(X + o1);
                dst[2] = *reinterpret_cast<const u32x4 *>(X + o2);
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
    auto stash = [&](int v, const u32x4 (&src)[3], const float (&sv)[2]) {
        uint8_t *Ls = &lds[v & 1][0];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            *reinterpret_cast<u32x4 *>(&Ls[(j * kDM + frow) * kDRow + fpart]) = src[j];
        const int i = v / nslices;
        if (v - i * nslices == 0 && tid < kDM + kDN) {
            tv[i & 1][0][tid] = sv[0];
            if (FP8) tv[i & 1][1][tid] = sv[1];
        }
    };
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    auto compute = [&](int buf) {
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
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bb[j], acc[i][j],
                                                                        0, 0, 0);
        }
    };
    // The distances of a finished tile (the arithmetic of the distance kernel's epilogue),
    // appended to the lists of their rows where they are within the rows' bounds.
    auto epilogue = [&](int i_tile) {
        const int n0 = (t0 + i_tile) * kDN;
        const float(&t)[2][kDM + kDN] = tv[i_tile & 1];
        // The lane's first row, made opaque here so that the compiler does not hoist the
        // 32 row addresses of the lists out of the tile loop (they would be spilled).
        int rbase = wm * 64 + 4 * half;
        asm volatile("" : "+v"(rbase));
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int rl0 = rbase + i * 32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rl = rl0 + 8 * (r >> 2) + (r & 3);
                const uint64_t B = s_bound[rl];
                const bool row_ok = m0 + rl < M;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int cl = wn * 64 + j * 32 + r32, col = n0 + cl;
                    const float xc = t[0][kDM + cl];
                    const float sc = FP8 ? t[1][kDM + cl] : 1.0f;
                    const float dot = FP8 ? (t[1][rl] * sc) * acc[i][j][r] : acc[i][j][r];
                    const float dv = (t[0][rl] + xc) - 2.0f * dot;
                    acc[i][j][r] = 0.f;
                    const uint64_t p = ((uint64_t)fkey(dv) << 32) | (uint32_t)col;
                    if (row_ok && col < N && p <= B) {
                        const uint32_t pos = atomicAdd(&s_cnt[rl], 1u);
                        Lb[(size_t)rl * kKnnCap + pos] = p;
                    }
                }
            }
        }
    };
    __syncthreads();
    if (U > 0) {
        fetch(0, pre, prv);
        stash(0, pre, prv);
        if (1 < U) fetch(1, pre, prv);
        __syncthreads();
    }
    int tile = 0, sl = 0;
    for (int u = 0; u < U; ++u) {
        compute(u & 1);
        if (u + 1 < U) {
            stash(u + 1, pre, prv);
            if (u + 2 < U) fetch(u + 2, pre, prv);
        }
        if (++sl == nslices) {
            epilogue(tile);
            __syncthreads();                       // every append of the tile is done
            for (int rl = wave; rl < kDM; rl += kDThreads / 64)
                if (s_cnt[rl] > (uint32_t)kKnnTrigger)
                    knn_compact(Lb + (size_t)rl * kKnnCap, &s_cnt[rl], &s_bound[rl], k, lane);
            ++tile;
            sl = 0;
        }
        __syncthreads();
    }
    // Last tightening (fewer entries for the merge), then the per-row results.
    for (int rl = wave; rl < kDM; rl += kDThreads / 64)
        if (s_cnt[rl] > (uint32_t)k)
            knn_compact(Lb + (size_t)rl * kKnnCap, &s_cnt[rl], &s_bound[rl], k, lane);
    __syncthreads();
    if (tid < kDM) {
        cnt_out[(size_t)b * kDM + tid] = s_cnt[tid];
        bound_out[(size_t)b * kDM + tid] = s_bound[tid];
    }
}

constexpr int kMergeThreads = 256;
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
    __shared__ uint32_t s_blk[kKnnMaxSplit], s_n[kKnnMaxSplit];
    __shared__ uint64_t s_B;
    __shared__ uint32_t s_gather, s_win, s_sel[3];
    const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int m = q / kDM, r = q % kDM;
    if (tid < nsplit) {
        const int s = tid;
        const uint32_t blk = (uint32_t)(kXcds * (m + mt * (s / kXcds)) + s % kXcds);
        s_blk[s] = blk;
        s_n[s] = cnt[(size_t)blk * kDM + r];
    }
    if (tid == 0) {
        s_gather = 0;
        s_win = 0;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t B = ~0ull;
        for (int s = 0; s < nsplit; ++s) {
            const uint64_t v = bound[(size_t)s_blk[s] * kDM + r];
            B = v < B ? v : B;
        }
        s_B = B;
    }
    __syncthreads();
    const uint64_t Bs = s_B;
    // Gather the entries <= B* into LDS while they fit.
    for (int s = 0; s < nsplit; ++s) {
        const uint64_t *L = lists + ((size_t)s_blk[s] * kDM + r) * kKnnCap;
        const int n = (int)s_n[s];
        for (int j = tid; j < n; j += kMergeThreads) {
            const uint64_t e = L[j];
            if (e <= Bs) {
                const uint32_t pos = atomicAdd(&s_gather, 1u);
                if (pos < (uint32_t)kMergeCap) buf[pos] = e;
            }
        }
    }
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
    uint64_t prefix = 0, mask = 0;
    uint32_t remaining = (uint32_t)kk;
    for (int pass = 0; pass < 8; ++pass) {
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
            for (int s = 0; s < nsplit; ++s) {
                const uint64_t *L = lists + ((size_t)s_blk[s] * kDM + r) * kKnnCap;
                const int n = (int)s_n[s];
                for (int j0 = 0; j0 < n; j0 += kMergeThreads) {
                    const int j = j0 + tid;
                    const uint64_t e = j < n ? L[j] : ~0ull;
                    const bool pend = j < n && e <= Bs && (e & mask) == prefix;
                    hist_add(hist, pend, (uint32_t)(e >> shift) & 255u, lane);
                }
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
        for (int s = 0; s < nsplit; ++s) {
            const uint64_t *L = lists + ((size_t)s_blk[s] * kDM + r) * kKnnCap;
            const int n = (int)s_n[s];
            for (int j = tid; j < n; j += kMergeThreads) {
                const uint64_t e = L[j];
                take(e, e <= Bs);
            }
        }
    }
    __syncthreads();
    // Sort the winners (padded to 256) ascending: bitonic, one element per thread.
    uint64_t v = tid < kk ? win[tid] : ~0ull;
    for (int size = 2; size <= kKnnMaxK; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            win[tid] = v;
            __syncthreads();
            const uint64_t o = win[tid ^ stride];
            const bool up = (tid & size) == 0, lower = (tid & stride) == 0;
            v = (lower == up) ? (o < v ? o : v) : (o > v ? o : v);
        }
    if (tid < k) {
        idx[(size_t)q * k + tid] = tid < kk ? (int32_t)(uint32_t)v : -1;
        dout[(size_t)q * k + tid] = tid < kk ? fkey_inv((uint32_t)(v >> 32)) : __int_as_float(0x7fc00000);
    }
}

// Direct-form squared distances of given pairs: d = sum_i (q_i - x_i)^2 over the stored
// (dequantised) values, summed in double and rounded once to float; exactly 0 for equal
// codes and scales. One wave per pair, four pairs per block.
template <bool FP8>
__global__ void __launch_bounds__(256) knn_direct_kernel(int M, int N, int k, int K,
                                                         const uint8_t *__restrict__ Q,
                                                         const float *__restrict__ qs,
                                                         const uint8_t *__restrict__ X,
                                                         const float *__restrict__ xs,
                                                         const int32_t *__restrict__ idx,
                                                         float *__restrict__ d)
{
    const int lane = threadIdx.x & 63;
    const int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pair >= (int64_t)M * k) return;
    const int q = (int)(pair / k);
    const int32_t e = idx[pair];
    if (e < 0 || e >= N) return;
    double acc = 0.0;
    if (FP8) {
        const double sq = qs[q], sx = xs[e];
        for (int i = lane; i < K; i += 64) {
            const double a = sq * (double)e4m3_val(Q[(int64_t)q * K + i]);
            const double c = sx * (double)e4m3_val(X[(int64_t)e * K + i]);
            acc += (a - c) * (a - c);
        }
    } else {
        const uint16_t *q16 = reinterpret_cast<const uint16_t *>(Q);
        const uint16_t *x16 = reinterpret_cast<const uint16_t *>(X);
        for (int i = lane; i < K; i += 64) {
            const double a = bf16_val(q16[(int64_t)q * K + i]);
            const double c = bf16_val(x16[(int64_t)e * K + i]);
            acc += (a - c) * (a - c);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) d[pair] = (float)acc;
}

// ---- launchers ----

int knn_splits(int M, int N)
{
    (void)M;
    const int nt = (N + kDN - 1) / kDN;
    const int ns = kXcds * (nt / (6 * kXcds));   // at least six tiles per split
    return max(kXcds, min(kKnnMaxSplit, ns));
}

size_t knn_ws_bytes(int M, int N)
{
    const size_t G = (size_t)((M + kDM - 1) / kDM) * knn_splits(M, N);
    return align_up(G * kDM * kKnnCap * 8, kAlign) + align_up(G * kDM * 4, kAlign) +
           align_up(G * kDM * 8, kAlign);
}

hipError_t launch_knn(bool fp8, int M, int N, int K, const void *Q, const float *qs,
                      const float *qn, const void *X, const float *xs, const float *xn, int k,
                      bool direct, int32_t *idx, float *d, void *ws, hipStream_t s)
{
    const int mt = (M + kDM - 1) / kDM, nsplit = knn_splits(M, N), nt = (N + kDN - 1) / kDN;
    const size_t G = (size_t)mt * nsplit;
    uint64_t *lists = static_cast<uint64_t *>(ws);
    char *p = static_cast<char *>(ws) + align_up(G * kDM * kKnnCap * 8, kAlign);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(p);
    uint64_t *bound = reinterpret_cast<uint64_t *>(p + align_up(G * kDM * 4, kAlign));
    const auto *q = static_cast<const uint8_t *>(Q);
    const auto *x = static_cast<const uint8_t *>(X);
    if (fp8)
        hipLaunchKernelGGL((knn_kernel<true, false>), dim3((unsigned)G), dim3(kDThreads), 0, s, M,
                           N, K, k, mt, nsplit, nt, q, qs, qn, x, xs, xn, lists, cnt, bound);
    else if ((2 * K) % kDSlice)
        hipLaunchKernelGGL((knn_kernel<false, true>), dim3((unsigned)G), dim3(kDThreads), 0, s, M,
                           N, K, k, mt, nsplit, nt, q, nullptr, qn, x, nullptr, xn, lists, cnt,
                           bound);
    else
        hipLaunchKernelGGL((knn_kernel<false, false>), dim3((unsigned)G), dim3(kDThreads), 0, s, M,
                           N, K, k, mt, nsplit, nt, q, nullptr, qn, x, nullptr, xn, lists, cnt,
                           bound);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)M), dim3(kMergeThreads), 0, s, k, mt,
                       nsplit, lists, cnt, bound, idx, d);
    e = hipGetLastError();
    if (e != hipSuccess || !direct) return e;
    const int64_t pairs = (int64_t)M * k;
    if (fp8)
        hipLaunchKernelGGL((knn_direct_kernel<true>), dim3((unsigned)((pairs + 3) / 4)), dim3(256),
                           0, s, M, N, k, K, q, qs, x, xs, idx, d);
    else
        hipLaunchKernelGGL((knn_direct_kernel<false>), dim3((unsigned)((pairs + 3) / 4)),
                           dim3(256), 0, s, M, N, k, K, q, nullptr, x, nullptr, idx, d);
    return hipGetLastError();
}

}  // namespace tdb
