// embed_core.hpp — pieces shared by the latent-distance kernels (embed.hip) and the
// fused distance + nearest-k kernels (knn.hip): vector types, the BF16 / e4m3 decoders,
// the tile shape of the LDS-staged distance GEMM and a wave-aggregated histogram add.
#pragma once

#include "common.hpp"

namespace tdb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float e4m3_val(uint8_t c)
{
    const int E = (c >> 3) & 15, m = c & 7;
    const float mag = E == 0 ? (float)m * 0.001953125f : ldexpf(1.0f + (float)m * 0.125f, E - 7);
    return (c & 0x80) ? -mag : mag;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Eight OCP e4m3 codes (bytes, lowest first) -> eight BF16 values (16 bytes, same order).
// gfx950's v_cvt_scalef32_pk_bf16_fp8 converts the two codes of one 16-bit word; with
// a scale of 1 the result is the code's value, which BF16 always holds exactly (its
// exponent range covers e4m3's normals and subnormals, its 8-bit significand the
// 4-bit one).
__device__ __forceinline__ u32x4 e4m3x8_to_bf16(u32x2 c)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c.x, 1.0f, false);
    const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c.x, 1.0f, true);
    const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c.y, 1.0f, false);
    const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c.y, 1.0f, true);
    return (u32x4){__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1),
                   __builtin_bit_cast(uint32_t, p2), __builtin_bit_cast(uint32_t, p3)};
}

// Distance GEMM tile: 128 queries x 256 database rows, K staged through LDS in slices of
// 64 bytes (32 BF16 values) per row, rows padded to 80 bytes; 512 threads (8 waves of
// 64 x 64). Blocks are placed on the 8 XCDs round robin (block b on XCD b % 8).
constexpr int kDM = 128, kDN = 256, kDSlice = 64, kDRow = 80, kDThreads = 512;
constexpr int kXcds = 8;

// LDS histogram increment for the pending lanes of a wave: a single add when
// they all fall into one bin (distances of a row are often concentrated, and
// same-address atomics serialise), else one atomic per lane.
__device__ __forceinline__ void hist_add(uint32_t *hist, bool pending, uint32_t bin, int lane)
{
    const uint64_t m = __ballot(pending);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const uint32_t b = __shfl(bin, leader, 64);
    if (__ballot(pending && bin != b) == 0) {
        if (lane == leader) atomicAdd(&hist[b], (uint32_t)__popcll(m));
    } else if (pending) {
        atomicAdd(&hist[bin], 1u);
    }
}

}  // namespace tdb
