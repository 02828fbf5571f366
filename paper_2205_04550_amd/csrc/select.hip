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
//  - k <= kSmallK: one wave per block. Each lane sorts kLaneR candidates in
//    registers (bitonic network, compile-time indices), then k rounds of a
//    64-lane arg-best (xor shuffles) pop the wave's k best.
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

__device__ __forceinline__ double entry_score(const TopkArgs &a, int q, int64_t e)
{
    const uint32_t *I = a.inter + q * a.inter_qstride + 2 * e;
    const uint32_t *B = a.bcnt + q * a.bcnt_qstride + 2 * e;
    const uint32_t *A = a.acnt + 2 * q;
    const double d_flair = dice(I[0], A[0], B[0]);
    const double d_t1 = dice(I[1], A[1], B[1]);
    return d_t1 + d_flair;
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
constexpr int kLaneR = 16;
constexpr int kWaveChunk = 64 * kLaneR;

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

// Sort kLaneR register pairs best first (bitonic network over xor partners).
__device__ __forceinline__ void sort_lane(uint64_t (&s)[kLaneR], int32_t (&ix)[kLaneR])
{
#pragma unroll
    for (int size = 2; size <= kLaneR; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < kLaneR; ++i) {
                const int j = i ^ stride;
                if (j > i)
                    order_pair(s[i], ix[i], s[j], ix[j], (i & size) == 0);
            }
}

template <bool FROM_COUNTS>
__global__ void __launch_bounds__(64) topk_wave_kernel(TopkArgs a, const uint64_t *src_s,
                                                       const int32_t *src_i, int64_t m, int nblk,
                                                       bool final_level, uint64_t *dst_s,
                                                       int32_t *dst_i)
{
    const int q = blockIdx.y;
    const int lane = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kWaveChunk;
    uint64_t s[kLaneR];
    int32_t ix[kLaneR];
#pragma unroll
    for (int r = 0; r < kLaneR; ++r) {
        const int64_t c = c0 + r * 64 + lane;
        if (c < m) {
            if (FROM_COUNTS) {
                s[r] = (uint64_t)__double_as_longlong(entry_score(a, q, c));
                ix[r] = (int32_t)c;
            } else {
                s[r] = src_s[(int64_t)q * m + c];
                ix[r] = src_i[(int64_t)q * m + c];
            }
        } else {
            s[r] = 0;        // padding ranks after every real entry
            ix[r] = INT_MAX;
        }
    }
    sort_lane(s, ix);
    const int64_t row = (int64_t)q * nblk + blockIdx.x;
    for (int r = 0; r < a.k; ++r) {
        uint64_t bs = s[0];
        int32_t bi = ix[0];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t os = __shfl_xor(bs, off, 64);
            const int32_t oi = __shfl_xor(bi, off, 64);
            if (ranks_before(os, oi, bs, bi)) {
                bs = os;
                bi = oi;
            }
        }
        if (lane == 0) {
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
        // The lane holding the winner pops it (indices are unique; equal
        // padding pairs may pop together, which leaves padding in place).
        if (s[0] == bs && ix[0] == bi) {
#pragma unroll
            for (int t = 0; t + 1 < kLaneR; ++t) {
                s[t] = s[t + 1];
                ix[t] = ix[t + 1];
            }
            s[kLaneR - 1] = 0;
            ix[kLaneR - 1] = INT_MAX;
        }
    }
}

// Blocks of the first selection level for n candidates per query, for sizing
// the candidate buffers: the wave path uses the smaller chunk, so it bounds both.
int64_t topk_blocks(int64_t n) { return (n + kWaveChunk - 1) / kWaveChunk; }

static int64_t bitonic_blocks(int64_t n) { return (n + kCH - 1) / kCH; }

static hipError_t launch_topk_small(const TopkArgs &a, hipStream_t s)
{
    int64_t m = a.n;
    int64_t nblk = (m + kWaveChunk - 1) / kWaveChunk;
    bool fin = nblk == 1;
    int cur = 0;
    hipLaunchKernelGGL((topk_wave_kernel<true>), dim3((unsigned)nblk, a.nq), dim3(64), 0, s, a,
                       nullptr, nullptr, m, (int)nblk, fin, a.buf_s[cur], a.buf_i[cur]);
    hipError_t err = hipGetLastError();
    m = nblk * a.k;
    while (!fin && err == hipSuccess) {
        nblk = (m + kWaveChunk - 1) / kWaveChunk;
        fin = nblk == 1;
        hipLaunchKernelGGL((topk_wave_kernel<false>), dim3((unsigned)nblk, a.nq), dim3(64), 0, s,
                           a, a.buf_s[cur], a.buf_i[cur], m, (int)nblk, fin, a.buf_s[cur ^ 1],
                           a.buf_i[cur ^ 1]);
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
