// select.hip — Dice, summed score and top-k of every query.
//
// Paper Sec. 2.3: Dice is the similarity of each mask; the two values are
// added (Dice_T1Gd + Dice_FLAIR) and the highest combined value is the best
// match. Dice_m = 2 I_m / (A_m + B_m) is evaluated in IEEE double (1 when
// both masks are empty), and entries are ranked by (score desc, index asc),
// a total order, so the result is unique.
//
// Selection is a tree: every block keeps the k best of its chunk of
// candidates; levels repeat on the survivors until one block per query
// remains, which writes the outputs.
//  - k <= kSmallK: four waves per block. Each lane sorts kLaneR candidates in
//    registers (bitonic network, compile-time indices); k rounds of a 64-lane
//    arg-best (DPP rotations within rows of 16, then two shuffles) pop each
//    wave's k best into LDS, and k more rounds on one wave pop the block's.
//  - larger k: 256 threads rank kTopkChunk candidates in LDS with a bitonic
//    network.
#include <limits.h>

#include "common.hpp"
#include "internal.hpp"

namespace tdb {

constexpr int kCH = kTopkChunk;

// Sort kCH (score bits, index) pairs in LDS, best first.
__device__ void bitonic_best_first(uint64_t *ks, int32_t *ki)
{
    for (int size = 2; size <= kCH; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < kCH / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t si = ks[i], sj = ks[j];
                const int32_t ii = ki[i], ij = ki[j];
                if (ranks_before(sj, ij, si, ii) == up) {
                    ks[i] = sj;
                    ks[j] = si;
                    ki[i] = ij;
                    ki[j] = ii;
                }
            }
        }
    }
    __syncthreads();
}

// Summed score from the counts of one (query, entry): [0] FLAIR, [1] T1Gd.
__device__ __forceinline__ double score_of(const uint32_t (&I)[2], const uint32_t (&A)[2],
                                           const uint32_t (&B)[2])
{
    const double d_flair = dice(I[0], A[0], B[0]);
    const double d_t1 = dice(I[1], A[1], B[1]);
    return d_t1 + d_flair;
}

__device__ __forceinline__ double entry_score(const TopkArgs &a, int q, int64_t e)
{
    const uint32_t *I = a.inter + q * a.inter_qstride + 2 * e;
    const uint32_t *B = a.bcnt + q * a.bcnt_qstride + 2 * e;
    const uint32_t *A = a.acnt + 2 * q;
    const uint32_t i2[2] = {I[0], I[1]}, a2[2] = {A[0], A[1]}, b2[2] = {B[0], B[1]};
    return score_of(i2, a2, b2);
}

__device__ void write_block(const TopkArgs &a, int q, bool final_level, int64_t out_row,
                            const uint64_t *ks, const int32_t *ki, uint64_t *dst_s, int32_t *dst_i)
{
    for (int r = threadIdx.x; r < a.k; r += blockDim.x) {
        if (final_level) {
            const int32_t e = ki[r];
            const int64_t o = (int64_t)q * a.k + r;
            a.out_idx[o] = e;
            a.out_score[o] = __longlong_as_double((long long)ks[r]);
            if (a.out_counts) {
                const uint32_t *I = a.inter + q * a.inter_qstride + 2 * (int64_t)e;
                const uint32_t *B = a.bcnt + q * a.bcnt_qstride + 2 * (int64_t)e;
                const uint32_t *A = a.acnt + 2 * q;
                db_counts_t c;
                c.inter[0] = I[0];
                c.inter[1] = I[1];
                c.a[0] = A[0];
                c.a[1] = A[1];
                c.b[0] = B[0];
                c.b[1] = B[1];
                a.out_counts[o] = c;
            }
        } else {
            dst_s[out_row * a.k + r] = ks[r];
            dst_i[out_row * a.k + r] = ki[r];
        }
    }
}

// Level 0: candidates are database entries; scores computed from counts.
// grid (blocks per query, nq). Output rows [q][blockIdx.x][k].
__global__ void __launch_bounds__(256) topk_first_kernel(TopkArgs a, int nblk, bool final_level,
                                                         uint64_t *dst_s, int32_t *dst_i)
{
    __shared__ uint64_t ks[kCH];
    __shared__ int32_t ki[kCH];
    const int q = blockIdx.y;
    const int64_t e0 = (int64_t)blockIdx.x * kCH;
    for (int t = threadIdx.x; t < kCH; t += blockDim.x) {
        const int64_t e = e0 + t;
        if (e < a.n) {
            ks[t] = (uint64_t)__double_as_longlong(entry_score(a, q, e));
            ki[t] = (int32_t)e;
        } else {
            ks[t] = 0;          // padding ranks after every real entry:
            ki[t] = INT_MAX;    // equal score bits (0.0) but a larger index
        }
    }
    bitonic_best_first(ks, ki);
    write_block(a, q, final_level, (int64_t)q * nblk + blockIdx.x, ks, ki, dst_s, dst_i);
}

// Later levels: candidates are (score bits, index) rows [q][m].
__global__ void __launch_bounds__(256) topk_merge_kernel(TopkArgs a, const uint64_t *src_s,
                                                         const int32_t *src_i, int64_t m,
                                                         int nblk, bool final_level,
                                                         uint64_t *dst_s, int32_t *dst_i)
{
    __shared__ uint64_t ks[kCH];
    __shared__ int32_t ki[kCH];
    const int q = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kCH;
    for (int t = threadIdx.x; t < kCH; t += blockDim.x) {
        const int64_t c = c0 + t;
        if (c < m) {
            ks[t] = src_s[(int64_t)q * m + c];
            ki[t] = src_i[(int64_t)q * m + c];
        } else {
            ks[t] = 0;
            ki[t] = INT_MAX;
        }
    }
    bitonic_best_first(ks, ki);
    write_block(a, q, final_level, (int64_t)q * nblk + blockIdx.x, ks, ki, dst_s, dst_i);
}

// ---- small k: register sort + wave arg-best rounds ---------------------------------------
constexpr int kSmallK = 32;
constexpr int kLaneR = 4;                          // candidates per lane
constexpr int kSelWaves = 4;                       // waves per block
constexpr int kSelChunk = 64 * kSelWaves * kLaneR; // candidates per block

__device__ __forceinline__ void order_pair(uint64_t &sa, int32_t &ia, uint64_t &sb, int32_t &ib,
                                           bool best_first)
{
    const bool b_first = ranks_before(sb, ib, sa, ia);
    if (b_first == best_first) {
        const uint64_t ts = sa;
        const int32_t ti = ia;
        sa = sb;
        ia = ib;
        sb = ts;
        ib = ti;
    }
}

// Sort R register pairs best first (bitonic network over xor partners).
template <int R>
__device__ __forceinline__ void sort_lane(uint64_t (&s)[R], int32_t (&ix)[R])
{
#pragma unroll
    for (int size = 2; size <= R; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int j = i ^ stride;
                if (j > i)
                    order_pair(s[i], ix[i], s[j], ix[j], (i & size) == 0);
            }
}

// The lane holding the winner (bs, bi) at the head of its sorted list pops it (indices
// are unique; equal padding pairs may pop together, which leaves padding in place).
template <int R>
__device__ __forceinline__ void pop_head(uint64_t (&s)[R], int32_t (&ix)[R], uint64_t bs,
                                         int32_t bi)
{
    if (s[0] == bs && ix[0] == bi) {
#pragma unroll
        for (int t = 0; t + 1 < R; ++t) {
            s[t] = s[t + 1];
            ix[t] = ix[t + 1];
        }
        s[R - 1] = 0;
        ix[R - 1] = INT_MAX;
    }
}

// One step of the wave's arg-best: take the partner's pair if it ranks before this lane's.
template <int CTRL>
__device__ __forceinline__ void best_step_dpp(uint64_t &bs, int32_t &bi)
{
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)bs);
    const uint32_t hi = dpp_u32<CTRL>((uint32_t)(bs >> 32));
    const int32_t oi = (int32_t)dpp_u32<CTRL>((uint32_t)bi);
    const uint64_t os = (uint64_t)hi << 32 | lo;
    if (ranks_before(os, oi, bs, bi)) {
        bs = os;
        bi = oi;
    }
}

// Every lane ends with the best (score, index) pair of the wave: rotations by 8, 4, 2
// and 1 within each row of 16 lanes (DPP), then exchanges with the lanes 16 and 32 away.
__device__ __forceinline__ void wave_best(uint64_t &bs, int32_t &bi)
{
    best_step_dpp<0x128>(bs, bi);   // row_ror 8
    best_step_dpp<0x124>(bs, bi);   // row_ror 4
    best_step_dpp<0x122>(bs, bi);   // row_ror 2
    best_step_dpp<0x121>(bs, bi);   // row_ror 1
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
        const uint64_t os = __shfl_xor(bs, off, 64);
        const int32_t oi = __shfl_xor(bi, off, 64);
        if (ranks_before(os, oi, bs, bi)) {
            bs = os;
            bi = oi;
        }
    }
}

// Rank r of the block's k best: the outputs at the last level, else a candidate row.
__device__ __forceinline__ void emit_best(const TopkArgs &a, int q, bool final_level,
                                          int64_t row, int r, uint64_t bs, int32_t bi,
                                          uint64_t *dst_s, int32_t *dst_i)
{
    if (final_level) {
        const int64_t o = (int64_t)q * a.k + r;
        a.out_idx[o] = bi;
        a.out_score[o] = __longlong_as_double((long long)bs);
        if (a.out_counts) {
            const uint32_t *I = a.inter + q * a.inter_qstride + 2 * (int64_t)bi;
            const uint32_t *B = a.bcnt + q * a.bcnt_qstride + 2 * (int64_t)bi;
            const uint32_t *A = a.acnt + 2 * q;
            db_counts_t c;
            c.inter[0] = I[0];
            c.inter[1] = I[1];
            c.a[0] = A[0];
            c.a[1] = A[1];
            c.b[0] = B[0];
            c.b[1] = B[1];
            a.out_counts[o] = c;
        }
    } else {
        dst_s[row * a.k + r] = bs;
        dst_i[row * a.k + r] = bi;
    }
}

// A block takes kSelChunk candidates of one query: each lane sorts its kLaneR in
// registers, each wave pops its k best into LDS by k arg-best rounds, and wave 0 pops
// the block's k best from those kSelWaves * k (at most two per lane).
template <bool FROM_COUNTS>
__global__ void __launch_bounds__(64 * kSelWaves) topk_block_kernel(
    TopkArgs a, const uint64_t *src_s, const int32_t *src_i, int64_t m, int nblk,
    bool final_level, uint64_t *dst_s, int32_t *dst_i)
{
    static_assert(kSelWaves * kSmallK <= 128, "the merge holds two candidates per lane");
    __shared__ uint64_t ls[kSelWaves * kSmallK];
    __shared__ int32_t li[kSelWaves * kSmallK];
    const int q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kSelChunk + threadIdx.x;
    uint64_t s[kLaneR];
    int32_t ix[kLaneR];
    // Every load is issued before any is used (addresses past the end are clamped to
    // candidate 0, m >= 1), so the lane waits for memory once, not once per candidate.
    if (FROM_COUNTS) {
        const uint32_t *I = a.inter + q * a.inter_qstride;
        const uint32_t *B = a.bcnt + q * a.bcnt_qstride;
        const uint32_t A[2] = {a.acnt[2 * q], a.acnt[2 * q + 1]};
        uint32_t iv[kLaneR][2], bv[kLaneR][2];
#pragma unroll
        for (int r = 0; r < kLaneR; ++r) {
            const int64_t c = c0 + r * 64 * kSelWaves;
            const int64_t e = c < m ? c : 0;
            iv[r][0] = I[2 * e];
            iv[r][1] = I[2 * e + 1];
            bv[r][0] = B[2 * e];
            bv[r][1] = B[2 * e + 1];
        }
#pragma unroll
        for (int r = 0; r < kLaneR; ++r) {
            s[r] = (uint64_t)__double_as_longlong(score_of(iv[r], A, bv[r]));
            ix[r] = (int32_t)(c0 + r * 64 * kSelWaves);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kLaneR; ++r) {
            const int64_t c = c0 + r * 64 * kSelWaves;
            const int64_t e = (int64_t)q * m + (c < m ? c : 0);
            s[r] = src_s[e];
            ix[r] = src_i[e];
        }
    }
#pragma unroll
    for (int r = 0; r < kLaneR; ++r) {
        if (c0 + r * 64 * kSelWaves >= m) {
            s[r] = 0;        // padding ranks after every real entry
            ix[r] = INT_MAX;
        }
    }
    sort_lane(s, ix);
    for (int r = 0; r < a.k; ++r) {
        uint64_t bs = s[0];
        int32_t bi = ix[0];
        wave_best(bs, bi);
        if (lane == 0) {
            ls[wave * kSmallK + r] = bs;
            li[wave * kSmallK + r] = bi;
        }
        pop_head(s, ix, bs, bi);
    }
    __syncthreads();
    if (wave != 0) return;
    uint64_t t[2];
    int32_t ti[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int j = lane + 64 * u;
        if (j < kSelWaves * a.k) {
            const int w = j / a.k;
            const int r = j - w * a.k;
            t[u] = ls[w * kSmallK + r];
            ti[u] = li[w * kSmallK + r];
        } else {
            t[u] = 0;
            ti[u] = INT_MAX;
        }
    }
    sort_lane(t, ti);
    // Lane r keeps the r-th winner; the k outputs (and, at the last level, their counts
    // loaded from memory) are then written by k lanes at once.
    uint64_t my_s = 0;
    int32_t my_i = INT_MAX;
    for (int r = 0; r < a.k; ++r) {
        uint64_t bs = t[0];
        int32_t bi = ti[0];
        wave_best(bs, bi);
        if (lane == r) {
            my_s = bs;
            my_i = bi;
        }
        pop_head(t, ti, bs, bi);
    }
    if (lane < a.k)
        emit_best(a, q, final_level, (int64_t)q * nblk + blockIdx.x, lane, my_s, my_i, dst_s,
                  dst_i);
}

// Blocks of the first selection level for n candidates per query, for sizing
// the candidate buffers: the wave path uses the smaller chunk, so it bounds both.
int64_t topk_blocks(int64_t n) { return (n + kSelChunk - 1) / kSelChunk; }

static int64_t bitonic_blocks(int64_t n) { return (n + kCH - 1) / kCH; }

static hipError_t launch_topk_small(const TopkArgs &a, hipStream_t s)
{
    int64_t m = a.n;
    int64_t nblk = (m + kSelChunk - 1) / kSelChunk;
    bool fin = nblk == 1;
    int cur = 0;
    hipLaunchKernelGGL((topk_block_kernel<true>), dim3((unsigned)nblk, a.nq), dim3(64 * kSelWaves),
                       0, s, a, nullptr, nullptr, m, (int)nblk, fin, a.buf_s[cur], a.buf_i[cur]);
    hipError_t err = hipGetLastError();
    m = nblk * a.k;
    while (!fin && err == hipSuccess) {
        nblk = (m + kSelChunk - 1) / kSelChunk;
        fin = nblk == 1;
        hipLaunchKernelGGL((topk_block_kernel<false>), dim3((unsigned)nblk, a.nq),
                           dim3(64 * kSelWaves), 0, s, a, a.buf_s[cur], a.buf_i[cur], m, (int)nblk,
                           fin, a.buf_s[cur ^ 1], a.buf_i[cur ^ 1]);
        err = hipGetLastError();
        cur ^= 1;
        m = nblk * a.k;
    }
    return err;
}

hipError_t launch_topk(const TopkArgs &a, hipStream_t s)
{
    if (a.k <= kSmallK)
        return launch_topk_small(a, s);
    int64_t nblk = bitonic_blocks(a.n);
    bool fin = nblk == 1;
    int cur = 0;
    hipLaunchKernelGGL(topk_first_kernel, dim3((unsigned)nblk, a.nq), dim3(256), 0, s, a,
                       (int)nblk, fin, a.buf_s[cur], a.buf_i[cur]);
    hipError_t err = hipGetLastError();
    int64_t m = nblk * a.k;
    while (!fin && err == hipSuccess) {
        nblk = bitonic_blocks(m);
        fin = nblk == 1;
        hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)nblk, a.nq), dim3(256), 0, s, a,
                           a.buf_s[cur], a.buf_i[cur], m, (int)nblk, fin, a.buf_s[cur ^ 1],
                           a.buf_i[cur ^ 1]);
        err = hipGetLastError();
        cur ^= 1;
        m = nblk * a.k;
    }
    return err;
}

}  // namespace tdb
