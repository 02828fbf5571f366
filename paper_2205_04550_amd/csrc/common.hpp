// common.hpp — device helpers shared by the retrieval kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdb {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Streaming 16-byte load that should not displace reused data (query words)
// from the caches: each database word is read exactly once per query.
__device__ __forceinline__ u32x4 load_stream(const u32x4 *p)
{
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ uint32_t popc(uint32_t x) { return (uint32_t)__builtin_popcount(x); }

// acc + popcount(x) as the single instruction the hardware has for it. Written out
// because the compiler otherwise pairs two popcounts into one three-way add, one
// instruction more per pair on count-bound loops.
__device__ __forceinline__ uint32_t popc_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

__device__ __forceinline__ uint32_t popc_and4(u32x4 a, u32x4 b)
{
    return popc(a.x & b.x) + popc(a.y & b.y) + popc(a.z & b.z) + popc(a.w & b.w);
}

__device__ __forceinline__ uint32_t popc4(u32x4 a)
{
    return popc(a.x) + popc(a.y) + popc(a.z) + popc(a.w);
}

// Bit 0 (FLAIR) and bit 1 (T1Gd) of the four label bytes of x as two nibbles
// (byte i -> bit i). Bytes 0..2 by one 24-bit multiply: with a = b0 + b1 2^8 +
// b2 2^16 (each 0 or 1), a * (2^16 + 2^9 + 2^2) holds b0, b1, b2 at bits 16..18,
// every other partial product on a distinct bit outside them (no carries); byte
// 3 by a shift.
__device__ __forceinline__ void label_nibbles(uint32_t x, uint32_t &n0, uint32_t &n1)
{
    const uint32_t a = x & 0x00010101u, b = (x >> 1) & 0x00010101u;
    n0 = ((__umul24(a, 0x010204u) >> 16) & 7u) | ((x >> 21) & 8u);
    n1 = ((__umul24(b, 0x010204u) >> 16) & 7u) | ((x >> 22) & 8u);
}

// Sum over the 64 lanes of a wave; every lane receives the total.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Sum over the bits set in word v of their positions 0..31: a position is the
// sum of its binary digits 2^j, so count, for every digit j, the set bits whose
// position has that digit.
__device__ __forceinline__ uint32_t bit_position_sum(uint32_t v)
{
    return popc(v & 0xAAAAAAAAu) + 2u * popc(v & 0xCCCCCCCCu) + 4u * popc(v & 0xF0F0F0F0u) +
           8u * popc(v & 0xFF00FF00u) + 16u * popc(v & 0xFFFF0000u);
}

// Order-preserving map of a float to uint32 (negative values flipped); -0 is
// folded onto +0 first so that equal values compare equal.
__device__ __forceinline__ uint32_t fkey(float f)
{
    if (f == 0.0f) f = 0.0f;
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float fkey_inv(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// One step of a radix select. counts[256] (LDS) holds the histogram of the
// current digit among the still-eligible keys; it is overwritten with its
// inclusive prefix sums, and the one thread whose bin holds the
// `remaining`-th smallest key writes out[0] = bin, out[1] = remaining minus
// the keys in lower bins. All threads of the block must call it (barriers);
// blockDim.x >= 256 and 1 <= remaining <= total count.
__device__ __forceinline__ void select_bin(uint32_t *counts, uint32_t remaining, uint32_t *out)
{
    const int t = threadIdx.x;
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = 0;
        if (t < 256 && t >= off) v = counts[t - off];
        __syncthreads();
        if (t < 256) counts[t] += v;
        __syncthreads();
    }
    if (t < 256) {
        const uint32_t incl = counts[t];
        const uint32_t excl = t ? counts[t - 1] : 0u;
        if (excl < remaining && incl >= remaining) {
            out[0] = (uint32_t)t;
            out[1] = remaining - excl;
        }
    }
    __syncthreads();
}

// Block-wide sum of two counters; the result is valid in thread 0.
// lds must hold 2 * (blockDim.x / 64) words.
__device__ __forceinline__ void block_sum2(uint32_t &a, uint32_t &b, uint32_t *lds)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    if (lane == 0) {
        lds[2 * wid] = a;
        lds[2 * wid + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + kWave - 1) / kWave;
        uint32_t sa = 0, sb = 0;
        for (int w = 0; w < nw; ++w) {
            sa += lds[2 * w];
            sb += lds[2 * w + 1];
        }
        a = sa;
        b = sb;
    }
}

// Dice of one mask in IEEE double; 1 when both masks are empty.
__device__ __forceinline__ double dice(uint32_t inter, uint32_t a, uint32_t b)
{
    uint64_t den = (uint64_t)a + (uint64_t)b;
    if (den == 0)
        return 1.0;
    return (double)(2 * (uint64_t)inter) / (double)den;
}

// Ranking order: higher score first, then lower index. Scores are
// non-negative doubles, so their bit patterns order like the values.
__device__ __forceinline__ bool ranks_before(uint64_t sa, int32_t ia, uint64_t sb, int32_t ib)
{
    return sa > sb || (sa == sb && ia < ib);
}

// v of the lane that DPP control `ctrl` names within this lane's row of 16 (all lanes active).
template <int ctrl>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, ctrl, 0xf, 0xf, false);
}

}  // namespace tdb
