// embed.hip — latent-distance search and exact-Dice rerank.
//
// Paper Sec. 2.3 ("Autoencoders"): the database and the query are encoded to
// latents and compared by L2 distance, lowest wins. Here the squared distance
// is expanded, d(q, x) = |q|^2 + |x|^2 - 2 q.x, so the dominant work is one
// dense contraction on the matrix cores, v_mfma_f32_32x32x16_bf16 with FP32
// accumulation, for both storage formats:
//   - BF16 latents are staged as they are;
//   - FP8 (OCP e4m3) latents with a per-row scale are decoded to BF16 while they
//     are staged into LDS (every e4m3 value is a BF16 value, so the decode is
//     exact); the products of the codes are then exact in FP32, and the scales
//     multiply the finished dot product.
// Each query keeps its k nearest latents, exactly, ties by lower index: a
// bound from per-chunk minima (the distance kernel can leave the minimum of
// every 16 consecutive entries for it) and a gather of the entries within the
// bound, or a radix select / chunked selection of the FP32 distances. Those
// candidates are re-scored with the exact Dice_T1Gd + Dice_FLAIR of the packed
// masks (Sec. 2.3 score), reading only the rows of the query's bounding box
// (outside it the query has no set bit, so those words add nothing to the
// overlap).
#include <limits.h>

#include "common.hpp"
#include "embed_core.hpp"
#include "internal.hpp"

namespace tdb {

// ---- quantisation ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}


// OCP FP8 e4m3 (bias 7, no infinities, largest finite 448): round to nearest
// even, saturating at +-448. Written from the format definition.
__device__ __forceinline__ uint8_t e4m3_rne(float v)
{
    const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
    float a = fabsf(v);
    if (!(a == a)) return (uint8_t)(sign | 0x7f);          // NaN
    if (a >= 448.0f) return (uint8_t)(sign | 0x7e);
    if (a < 0.015625f) {                                    // below 2^-6: subnormal step 2^-9
        const int m = (int)rintf(a * 512.0f);               // 0..8 (8 = smallest normal)
        return (uint8_t)(sign | (uint32_t)m);
    }
    int e;
    const float fr = frexpf(a, &e);                         // a = fr * 2^e, fr in [0.5, 1)
    int m = (int)rintf((fr * 2.0f - 1.0f) * 8.0f);          // exact scaling, then RNE
    int E = e - 1 + 7;
    if (m == 8) {
        m = 0;
        E += 1;
    }
    uint32_t code = ((uint32_t)E << 3) | (uint32_t)m;
    if (code > 0x7e) code = 0x7e;
    return (uint8_t)(sign | code);
}

// One block (256 threads) per row: BF16 copy and |x|^2 of the stored values.
__global__ void __launch_bounds__(256) quant_bf16_kernel(int dim, const float *__restrict__ x,
                                                         uint16_t *__restrict__ y,
                                                         float *__restrict__ sq)
{
    __shared__ double red[4];
    const int64_t r = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < dim; i += blockDim.x) {
        const uint16_t b = bf16_rne(x[r * dim + i]);
        y[r * dim + i] = b;
        const double v = bf16_val(b);
        acc += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sq[r] = (float)(((red[0] + red[1]) + red[2]) + red[3]);
}

// One block per row: scale s = max|x| / 448 (1 for a zero row), codes e4m3(x / s),
// |s * e4m3_val(code)|^2 summed in double.
__global__ void __launch_bounds__(256) quant_fp8_kernel(int dim, const float *__restrict__ x,
                                                        uint8_t *__restrict__ y,
                                                        float *__restrict__ scale,
                                                        float *__restrict__ sq)
{
    __shared__ float redm[4];
    __shared__ double red[4];
    const int64_t r = blockIdx.x;
    float amax = 0.f;
    for (int i = threadIdx.x; i < dim; i += blockDim.x) amax = fmaxf(amax, fabsf(x[r * dim + i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3]));
    const float s = amax > 0.f ? amax / 448.0f : 1.0f;
    double acc = 0.0;
    for (int i = threadIdx.x; i < dim; i += blockDim.x) {
        const uint8_t c = e4m3_rne(x[r * dim + i] / s);
        y[r * dim + i] = c;
        const double v = (double)s * (double)e4m3_val(c);
        acc += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        sq[r] = (float)(((red[0] + red[1]) + red[2]) + red[3]);
        scale[r] = s;
    }
}

// ---- distance GEMM, LDS-staged ----------------------------------------------------------------
//
// Tile 128 queries x 256 database rows, 8 waves as 2 x 4 of 64 x 64 (2 x 2 MFMA
// 32x32 tiles each). K is staged through LDS in slices of 64 bytes (32 bf16 or
// 64 fp8 values) for both operands, double-buffered, so each operand row is
// read from L2 once per tile instead of once per wave. LDS rows are padded to
// 80 bytes to spread the 16-byte fragment reads over the banks.
//
// The grid is persistent: block b of G (G a multiple of 8) takes the virtual
// tiles b, b + G, b + 2G, ..., and the K slices of all its tiles form one
// stream, loaded DEPTH slices ahead into a ring of registers. The loads of the
// next tile are in flight while the current one finishes and writes its
// distances, and DEPTH slices of load latency are covered instead of one.
// Virtual tiles are numbered so that consecutive numbers go to different XCDs
// (block b runs on XCD b % 8, and so do all its tiles): the blocks of one XCD
// work on a few database tiles at a time with every query tile, so a database
// tile comes from HBM into that XCD's L2 once and is reused there.
// Row offsets into Q and X are 32-bit: the host splits X into chunks below this.
constexpr int64_t kDChunkBytes = (int64_t)1 << 31;

// fkey without its folding of -0 onto +0 (three instructions instead of five): the same
// order, except that -0 sorts just below +0. The minimum of a set under raw_key, passed
// through fold_zero_key, is the minimum under fkey.
__device__ __forceinline__ uint32_t raw_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}
__device__ __forceinline__ uint32_t fold_zero_key(uint32_t k)
{
    return k == 0x7fffffffu ? 0x80000000u : k;   // raw_key(-0) -> fkey(+0)
}

// Reduce-scatter of minima over each row of 16 lanes: lane l returns the minimum of
// k[l % 16] over the 16 lanes of its row. Four exchange steps (row mirror, half-row
// mirror, xor 2, xor 1); in each a lane keeps the half of its values that the lane
// bit of that step selects and sends the other half to its partner.
__device__ __forceinline__ uint32_t row16_min_scatter(const uint32_t (&k)[16], int lane)
{
    const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
    uint32_t k1[8], k2[4], k3[2];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        k1[q] = min(b3 ? k[q + 8] : k[q], dpp_u32<0x140>(b3 ? k[q] : k[q + 8]));      // mirror
#pragma unroll
    for (int q = 0; q < 4; ++q)
        k2[q] = min(b2 ? k1[q + 4] : k1[q], dpp_u32<0x141>(b2 ? k1[q] : k1[q + 4]));  // half mirror
#pragma unroll
    for (int q = 0; q < 2; ++q)
        k3[q] = min(b1 ? k2[q + 2] : k2[q], dpp_u32<0x4e>(b1 ? k2[q] : k2[q + 2]));   // xor 2
    return min(b0 ? k3[1] : k3[0], dpp_u32<0xb1>(b0 ? k3[0] : k3[1]));                // xor 1
}

// GMIN: also write, for every row and every whole group of 16 consecutive columns
// g < ngroups, the smallest order key (fkey) of the group's distances to
// gmin[row * gld + g]; the bound of the top-k selection below then reads these
// instead of the distances (mode 0 only). With GMIN, D may be null: then only the
// minima are written.
template <bool FP8, bool TAIL, int DEPTH, bool GMIN>
__global__ void __launch_bounds__(kDThreads, 4) dist_lds_kernel(int M, int N, int K, int mt,
                                                             int ntiles,
                                                             const uint8_t *__restrict__ Q,
                                                             const float *__restrict__ qs,
                                                             const float *__restrict__ qn,
                                                             const uint8_t *__restrict__ X,
                                                             const float *__restrict__ xs,
                                                             const float *__restrict__ xn,
                                                             float *__restrict__ D, int64_t ldd,
                                                             int mode, uint32_t *__restrict__ gmin,
                                                             int64_t gld, int ngroups)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][(kDM + kDN) * kDRow];
    // Squared norms (and FP8 scales) of the rows of a tile, by tile parity:
    // [0..127] query rows, [128..383] database rows.
    __shared__ float tv[2][2][kDM + kDN];
    const int G = gridDim.x, b = blockIdx.x;
    const int Kb = FP8 ? K : 2 * K;                 // bytes per row in Q and X
    const int nslices = (2 * K + kDSlice - 1) / kDSlice;   // 32 values per slice
    const int mytiles = b < ntiles ? (ntiles - 1 - b) / G + 1 : 0;
    const int U = mytiles * nslices;                // K slices this block streams
    if (U == 0) return;                             // whole block, before any barrier
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    const int half = lane >> 5, r32 = lane & 31;
    // Origin of the i-th tile of this block. A virtual tile past the last
    // database tile (nt not a multiple of 8) has n0 >= N: its loads are clamped
    // to the last row and it stores nothing.
    auto origin = [&](int i, int &m0, int &n0) {
        const int p = b + i * G, q = p / kXcds;
        m0 = (q % mt) * kDM;
        n0 = ((q / mt) * kXcds + p % kXcds) * kDN;
    };
    // Staging: 384 rows x 4 chunks of 16 bytes, 3 chunks per thread: chunk
    // tid % 4 of query row tid / 4 and of database rows tid / 4 and 128 + tid / 4.
    // With the first slice of a tile, threads 0..383 also load the norm (and
    // scale) of row tid of the tile; they travel through the ring into tv
    // (loads issued at the epilogue would wait for every load in flight, as the
    // vector memory counter is in order).
    const int frow = tid >> 2, fpart = (tid & 3) * 16;
    u32x4 pre[DEPTH][3];
    float prv[DEPTH][2];
    auto fetch = [&](int v, u32x4 (&dst)[3], float (&dv)[2]) {
        const int i = v / nslices, sl = v - i * nslices;
        int m0, n0;
        origin(i, m0, n0);
        // Byte offset of this thread's 8 values (FP8) or 16 bytes (BF16) in its rows.
        const uint32_t kb = FP8 ? (uint32_t)(sl * (kDSlice / 2) + (fpart >> 1))
                                : (uint32_t)(sl * kDSlice + fpart);
        if (!TAIL || (int)kb < Kb) {
            const uint32_t o0 = (uint32_t)min(m0 + frow, M - 1) * (uint32_t)Kb + kb;
            const uint32_t o1 = (uint32_t)min(n0 + frow, N - 1) * (uint32_t)Kb + kb;
            const uint32_t o2 = (uint32_t)min(n0 + kDM + frow, N - 1) * (uint32_t)Kb + kb;
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
        uint8_t *L = &lds[v & 1][0];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            *reinterpret_cast<u32x4 *>(&L[(j * kDM + frow) * kDRow + fpart]) = src[j];
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
        const uint8_t *A = &lds[buf][0], *B = &lds[buf][kDM * kDRow];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(
                    A + (wm * 64 + i * 32 + r32) * kDRow + st * 32 + half * 16);
                b[i] = *reinterpret_cast<const bf16x8 *>(
                    B + (wn * 64 + i * 32 + r32) * kDRow + st * 32 + half * 16);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j],
                                                                        0, 0, 0);
        }
    };
    // Epilogue. mode 0: D = d (squared L2); mode 1: D = sqrt(max(d, 0)) (L2);
    // mode 2: D += sqrt(max(d, 0)) (a second L2 added to the first: the paper's
    // L2_T1Gd + L2_FLAIR of two encoders, Sec. 2.3).
    auto epilogue = [&](int i_tile) {
        int m0, n0;
        origin(i_tile, m0, n0);
        const float(&t)[2][kDM + kDN] = tv[i_tile & 1];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int cl = wn * 64 + j * 32 + r32, col = n0 + cl;
                const int rl0 = wm * 64 + i * 32 + 4 * half;
                const float xc = t[0][kDM + cl];
                const float sc = FP8 ? t[1][kDM + cl] : 1.0f;
                float *out = D + (int64_t)(m0 + rl0) * ldd + col;
                // No D (group minima only): nothing is stored.
                const int rows = col < N && D ? M - (m0 + rl0) : 0;
                uint32_t key[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int rr = 8 * (r >> 2) + (r & 3), rl = rl0 + rr;
                    const float dot = FP8 ? (t[1][rl] * sc) * acc[i][j][r] : acc[i][j][r];
                    const float dv = (t[0][rl] + xc) - 2.0f * dot;
                    if (rr < rows) {
                        // Non-temporal: the distances stream past L2, where the
                        // database tiles are meant to stay.
                        if (mode == 0) __builtin_nontemporal_store(dv, &out[rr * ldd]);
                        else {
                            const float l = __builtin_sqrtf(fmaxf(dv, 0.0f));
                            __builtin_nontemporal_store(mode == 1 ? l : out[rr * ldd] + l,
                                                        &out[rr * ldd]);
                        }
                    }
                    key[r] = col < N ? raw_key(dv) : 0xffffffffu;
                    acc[i][j][r] = 0.f;
                }
                if (GMIN) {                   // all 64 lanes active: DPP reads whole rows
                    const uint32_t gm = fold_zero_key(row16_min_scatter(key, lane));   // row rl0 + rr(lane % 16)
                    const int rr = 8 * ((lane & 15) >> 2) + (lane & 3);
                    const int g = (n0 + wn * 64 + j * 32 + (lane & 16)) >> 4;
                    if (m0 + rl0 + rr < M && g < ngroups)
                        gmin[(int64_t)(m0 + rl0 + rr) * gld + g] = gm;
                }
            }
    };
    // Ring invariant: slot s holds the slice of step v with v % DEPTH == s, for
    // the steps u + 1 .. u + DEPTH while step u is multiplied.
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
        if (d < U) fetch(d, pre[d], prv[d]);
    stash(0, pre[0], prv[0]);
    if (DEPTH < U) fetch(DEPTH, pre[0], prv[0]);
    __syncthreads();
    int tile = 0, sl = 0;
    for (int u0 = 0; u0 < U; u0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const int u = u0 + d;
            if (u < U) {
                compute(u & 1);
                if (u + 1 < U) {
                    const int nx = (d + 1) % DEPTH;
                    stash(u + 1, pre[nx], prv[nx]);
                    if (u + 1 + DEPTH < U) fetch(u + 1 + DEPTH, pre[nx], prv[nx]);
                }
                if (++sl == nslices) {
                    epilogue(tile);
                    ++tile;
                    sl = 0;
                }
                __syncthreads();
            }
        }
    }
}

// ---- exact k smallest per row (radix select) ----------------------------------------------

constexpr int kSelThreads = 1024;
constexpr int kSelMaxK = 1024;

// grid M, kSelThreads threads. Four 8-bit digit passes find the key T of the
// k-th smallest element; entries with key < T are taken, then the lowest
// indices among key == T; the k winners are sorted by (key, index).
__device__ __forceinline__ void select_row_radix(const float *__restrict__ row, int N, int k,
                                                 int32_t *__restrict__ oidx, float *__restrict__ od)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_sel[2];
    __shared__ uint32_t scan[kSelThreads];
    __shared__ uint32_t sk[kSelMaxK];
    __shared__ int32_t si[kSelMaxK];
    __shared__ uint32_t s_lt;
    const int lane = threadIdx.x & 63;
    uint32_t prefix = 0, mask = 0, remaining = (uint32_t)k;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        for (int base = 0; base < N; base += blockDim.x) {
            const int i = base + threadIdx.x;
            bool pending = false;
            uint32_t bin = 0;
            if (i < N) {
                const uint32_t u = fkey(row[i]);
                pending = (u & mask) == prefix;
                bin = (u >> shift) & 255u;
            }
            hist_add(hist, pending, bin, lane);
        }
        __syncthreads();
        select_bin(hist, remaining, s_sel);
        prefix |= s_sel[0] << shift;
        remaining = s_sel[1];
        mask |= 255u << shift;
        __syncthreads();
    }
    const uint32_t T = prefix;          // key of the k-th smallest
    const uint32_t n_lt = (uint32_t)k - remaining;
    // Entries below T (order fixed by the sort below) and per-thread counts of T in
    // contiguous index chunks.
    if (threadIdx.x == 0) s_lt = 0;
    __syncthreads();
    const int C = (N + blockDim.x - 1) / blockDim.x;
    const int c0 = threadIdx.x * C, c1 = min(N, c0 + C);
    uint32_t eq = 0;
    for (int i = c0; i < c1; ++i) {
        const uint32_t u = fkey(row[i]);
        if (u < T) {
            const uint32_t slot = atomicAdd(&s_lt, 1u);
            sk[slot] = u;
            si[slot] = i;
        } else if (u == T) {
            ++eq;
        }
    }
    scan[threadIdx.x] = eq;
    __syncthreads();
    // Exclusive prefix of the equal-key counts in index order (Hillis-Steele).
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t rank = scan[threadIdx.x] - eq;
    if (rank < remaining) {
        for (int i = c0; i < c1 && rank < remaining; ++i) {
            if (fkey(row[i]) == T) {
                sk[n_lt + rank] = T;
                si[n_lt + rank] = i;
                ++rank;
            }
        }
    }
    // Sort the k winners by (key, index); pad to a power of two.
    int P = 1;
    while (P < k) P <<= 1;
    for (int t = k + threadIdx.x; t < P; t += blockDim.x) {
        sk[t] = 0xffffffffu;
        si[t] = INT_MAX;
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint32_t ki = sk[i], kj = sk[j];
                const int32_t ii = si[i], ij = si[j];
                const bool j_first = kj < ki || (kj == ki && ij < ii);
                if (j_first == up) {
                    sk[i] = kj;
                    sk[j] = ki;
                    si[i] = ij;
                    si[j] = ii;
                }
            }
        }
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        oidx[t] = si[t];
        od[t] = fkey_inv(sk[t]);
    }
}

__global__ void __launch_bounds__(kSelThreads) topk_min_kernel(const float *__restrict__ D, int N,
                                                               int k, int32_t *__restrict__ out_idx,
                                                               float *__restrict__ out_d)
{
    const int64_t r = blockIdx.x;
    select_row_radix(D + r * N, N, k, out_idx + r * k, out_d + r * k);
}

// ---- exact rerank ---------------------------------------------------------------------------

constexpr int kRerankMaxCand = 1024;

constexpr int kRC = 4;                 // candidates per wave
static_assert(kRC == 4, "the LDS staging of the per-slice ranges picks among four members");
constexpr int kRerankPerBlock = 4 * kRC;   // candidates scored per block (4 waves)
constexpr int kZStage = 128;           // z-slices of per-slice row ranges a wave stages in LDS

// 1-D grid of nbq * 8 * ceil(nq / 8) blocks (nbq = ceil(count / candidates per block): 4 kRC,
// or kRC with SPLIT = 4), 256 threads (4 waves). Blocks go to the 8 XCDs round-robin; the mapping below
// gives every block of query q to XCD q % 8, so the query's rows are fetched into
// one L2 only. Each wave scores
// kRC candidates of query q at once: lanes sweep the rows where the query's row
// boxes meet the candidates' stored row boxes (outside either box one side is
// zero and adds nothing; the T1Gd plane has boxes of its own, smaller than those
// of both masks), AND + popcount against each candidate's planes; the score and
// overlaps go to ws (score bits [nq][nc], index [nq][nc], I [nq][nc][2]).
// SPLIT = 4: a block scores kRC candidates (not 4 kRC), its four waves taking every fourth
// pass over the rows and adding their overlaps in LDS: four times the waves per candidate, for
// launches with few candidates per query. ALLZR: nz <= kZStage, so every query's slices have
// their ranges staged.
template <int SPLIT, bool ALLZR>
__global__ void __launch_bounds__(256) rerank_score_kernel(const uint32_t *__restrict__ planes,
                                                           const uint32_t *__restrict__ popcnt,
                                                           const int32_t *__restrict__ ebox,
                                                           const int32_t *__restrict__ etbox,
                                                           const uint32_t *__restrict__ zrange,
                                                           int nz, int Wp,
                                                           int nxw, int ny,
                                                           const uint32_t *__restrict__ qpack,
                                                           const uint32_t *__restrict__ acnt,
                                                           const int32_t *__restrict__ box,
                                                           const int32_t *__restrict__ tbox,
                                                           const int32_t *__restrict__ cand, int nc,
                                                           uint64_t *__restrict__ ws_s,
                                                           int32_t *__restrict__ ws_i,
                                                           uint32_t *__restrict__ ws_I, int nq,
                                                           int nbq,
                                                           const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ ents,
                                                           const int32_t *__restrict__ qcount,
                                                           int first, int count)
{
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const int q = (slot / nbq) * 8 + xcd, qb = slot % nbq;
    if (q >= nq) return;                       // whole block, before any barrier
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t *Q0 = qpack + (int64_t)q * 2 * Wp, *Q1 = Q0 + Wp;
    const int32_t *b = box + 4 * q, *tb = tbox + 4 * q;
    const int qz0 = b[0], qz1 = b[1], qy0 = b[2], qy1 = b[3];
    const int tqz0 = tb[0], tqz1 = tb[1], tqy0 = tb[2], tqy1 = tb[3];
    const uint32_t A0 = acnt[2 * q], A1 = acnt[2 * q + 1];
    // kRC candidates per wave: each query row is loaded once per group, and the group sweeps
    // the union of its members' boxes. A member reads its FLAIR rows inside (its row box n the
    // query's) and its T1Gd rows inside (its T1Gd box n the query's): outside either pair of
    // boxes one of the two masks is empty.
    // This wave's candidates: positions first + c0 .. + kRC - 1 of the query's list, count of
    // them (qcount: the query's own count). With order, position i is slot order[i] and entry
    // ents[i] (the candidates in bound order); else slot = position.
    const int c0 = SPLIT == 1 ? qb * kRerankPerBlock + wave * kRC : qb * kRC;
    const int64_t qo = (int64_t)q * nc;
    const int cnt = qcount ? qcount[q] : count;
    int cs[kRC];
    int32_t ent[kRC];
    bool act[kRC], any = false;
#pragma unroll
    for (int j = 0; j < kRC; ++j) {
        const int i = first + c0 + j;
        act[j] = c0 + j < cnt && i < nc;
        const int ii = act[j] ? i : 0;
        cs[j] = order ? order[qo + ii] : ii;
        ent[j] = ents ? ents[qo + ii] : cand[qo + cs[j]];
        any |= act[j];
    }
    if (!any) return;       // a whole wave leaves; no block barrier below
    // Each member's per-slice y-ranges of its FLAIR and T1Gd rows over the query's slices (every
    // slice swept lies in them), in this wave's part of LDS, their loads issued together and
    // before the members' boxes are known (a query deeper than kZStage slices goes by the
    // boxes alone).
    __shared__ uint2 s_zr[4][kRC][kZStage];
    const int nzs = qz1 - qz0;
    const bool zr_ok = nzs > 0 && nzs <= kZStage;
    if (zr_ok) {
        constexpr int kStageMax = kRC * kZStage / 64;
        uint2 t[kStageMax];
#pragma unroll
        for (int u = 0; u < kStageMax; ++u) {
            const int i = lane + 64 * u, j = i / nzs, zz = i - j * nzs;
            const int32_t e = j == 0 ? ent[0] : j == 1 ? ent[1] : j == 2 ? ent[2] : ent[3];
            t[u] = i < kRC * nzs ? *reinterpret_cast<const uint2 *>(zrange + ((int64_t)e * nz + qz0 + zz) * 2)
                                 : (uint2){0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < kStageMax; ++u) {
            const int i = lane + 64 * u, j = i / nzs, zz = i - j * nzs;
            if (i < kRC * nzs) s_zr[wave][j][zz] = t[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const uint32_t *D0[kRC], *D1[kRC];
    int z0[kRC], z1[kRC], y0[kRC], y1[kRC], tz0[kRC], tz1[kRC], ty0[kRC], ty1[kRC];
    int uz0 = INT_MAX, uz1 = INT_MIN, uy0 = INT_MAX, uy1 = INT_MIN;
#pragma unroll
    for (int j = 0; j < kRC; ++j) {
        const int32_t e = ent[j];             // an inactive member sweeps no rows
        D0[j] = planes + (int64_t)e * 2 * Wp;
        D1[j] = D0[j] + Wp;
        const int32_t *eb = ebox + 4 * (int64_t)e, *etb = etbox + 4 * (int64_t)e;
        z0[j] = act[j] ? max(eb[0], qz0) : 0;
        z1[j] = act[j] ? min(eb[1], qz1) : 0;
        y0[j] = max(eb[2], qy0);
        y1[j] = min(eb[3], qy1);
        tz0[j] = act[j] ? max(etb[0], tqz0) : 0;
        tz1[j] = act[j] ? min(etb[1], tqz1) : 0;
        ty0[j] = max(etb[2], tqy0);
        ty1[j] = min(etb[3], tqy1);
        if (z1[j] > z0[j] && y1[j] > y0[j]) {
            uz0 = min(uz0, z0[j]);
            uz1 = max(uz1, z1[j]);
            uy0 = min(uy0, y0[j]);
            uy1 = max(uy1, y1[j]);
        }
        if (tz1[j] > tz0[j] && ty1[j] > ty0[j]) {
            uz0 = min(uz0, tz0[j]);
            uz1 = max(uz1, tz1[j]);
            uy0 = min(uy0, ty0[j]);
            uy1 = max(uy1, ty1[j]);
        }
    }
    const int nyr = uy1 > uy0 ? uy1 - uy0 : 0;
    const int nr = uz1 > uz0 ? (uz1 - uz0) * nyr : 0;
    // Row (z, y) of member j holds FLAIR bits only if y is in its FLAIR range of slice z.
    auto in_range = [&](int j, int z, int y, bool t1gd) {
        if (!zr_ok) return true;
        const uint2 rg = s_zr[wave][j][z - qz0];
        const uint32_t v = t1gd ? rg.y : rg.x;
        return y >= (int)(v & 0xffffu) && y < (int)(v >> 16);
    };
    uint32_t i0[kRC], i1[kRC];
#pragma unroll
    for (int j = 0; j < kRC; ++j) i0[j] = i1[j] = 0;
    if (nxw == 4) {
        // Rows of 128 voxels: one 16-byte load per plane; two rows per lane per pass, all
        // loads of the pass issued before any is used.
        constexpr int U = SPLIT == 1 ? 2 : 1;
        const int rw = SPLIT == 1 ? 0 : wave;
        for (int r0 = lane + 64 * U * rw; r0 < nr; r0 += 64 * U * SPLIT) {
            u32x4 qa[U], qb[U], da[U][kRC], db[U][kRC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = r0 + 64 * u;
                const int zr = r / nyr;
                const int z = uz0 + zr, y = uy0 + r - zr * nyr;
                const int base = (z * ny + y) * 4;
                const bool live = r < nr;
                bool any0 = false, any1 = false;
                // With the slice ranges staged, a member's range of a slice lies in its own row
                // boxes and the sweep in the query's row box: the range decides for FLAIR, the
                // range and the query's T1Gd box for T1Gd.
                const bool tin = z >= tqz0 && z < tqz1 && y >= tqy0 && y < tqy1;
#pragma unroll
                for (int j = 0; j < kRC; ++j) {
                    bool in0, in1;
                    if constexpr (ALLZR) {
                        in0 = live && act[j] && in_range(j, z, y, false);
                        in1 = live && act[j] && tin && in_range(j, z, y, true);
                    } else {
                        in0 = live && z >= z0[j] && z < z1[j] && y >= y0[j] && y < y1[j] &&
                              in_range(j, z, y, false);
                        in1 = live && z >= tz0[j] && z < tz1[j] && y >= ty0[j] && y < ty1[j] &&
                              in_range(j, z, y, true);
                    }
                    any0 |= in0;
                    any1 |= in1;
                    da[u][j] = db[u][j] = (u32x4){0u, 0u, 0u, 0u};
                    if (in0) da[u][j] = load_stream(reinterpret_cast<const u32x4 *>(D0[j] + base));
                    if (in1) db[u][j] = load_stream(reinterpret_cast<const u32x4 *>(D1[j] + base));
                }
                qa[u] = qb[u] = (u32x4){0u, 0u, 0u, 0u};
                if (any0) qa[u] = *reinterpret_cast<const u32x4 *>(Q0 + base);
                if (any1) qb[u] = *reinterpret_cast<const u32x4 *>(Q1 + base);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < kRC; ++j) {
                    i0[j] += popc_and4(qa[u], da[u][j]);
                    i1[j] += popc_and4(qb[u], db[u][j]);
                }
        }
    } else {
        for (int r = lane + (SPLIT == 1 ? 0 : 64 * wave); r < nr; r += 64 * SPLIT) {
            const int zr = r / nyr;
            const int z = uz0 + zr, y = uy0 + r - zr * nyr;
            const int base = (z * ny + y) * nxw;
            bool in0[kRC], in1[kRC];
#pragma unroll
            for (int j = 0; j < kRC; ++j) {
                in0[j] = z >= z0[j] && z < z1[j] && y >= y0[j] && y < y1[j] && in_range(j, z, y, false);
                in1[j] = z >= tz0[j] && z < tz1[j] && y >= ty0[j] && y < ty1[j] && in_range(j, z, y, true);
            }
            for (int w = 0; w < nxw; ++w) {
                const uint32_t qa = Q0[base + w], qb = Q1[base + w];
#pragma unroll
                for (int j = 0; j < kRC; ++j) {
                    if (in0[j]) i0[j] += popc(qa & D0[j][base + w]);
                    if (in1[j]) i1[j] += popc(qb & D1[j][base + w]);
                }
            }
        }
    }
    if constexpr (SPLIT > 1) {                // the four waves' overlaps, added in wave 0
        __shared__ uint32_t s_red[4][kRC][2];
#pragma unroll
        for (int j = 0; j < kRC; ++j) {
            const uint32_t a0 = wave_sum(i0[j]), a1 = wave_sum(i1[j]);
            if (lane == 0) {
                s_red[wave][j][0] = a0;
                s_red[wave][j][1] = a1;
            }
        }
        __syncthreads();
        if (wave) return;
#pragma unroll
        for (int j = 0; j < kRC; ++j) {
            i0[j] = lane == 0 ? s_red[0][j][0] + s_red[1][j][0] + s_red[2][j][0] + s_red[3][j][0] : 0u;
            i1[j] = lane == 0 ? s_red[0][j][1] + s_red[1][j][1] + s_red[2][j][1] + s_red[3][j][1] : 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < kRC; ++j) {
        const uint32_t a0 = wave_sum(i0[j]), a1 = wave_sum(i1[j]);
        if (lane == 0 && act[j]) {
            const int64_t o = qo + cs[j];
            const int32_t e = ent[j];
            const double sc = dice(a1, A1, popcnt[2 * (int64_t)e + 1]) +
                              dice(a0, A0, popcnt[2 * (int64_t)e]);
            ws_s[o] = (uint64_t)__double_as_longlong(sc);
            ws_i[o] = e;
            ws_I[2 * o] = a0;
            ws_I[2 * o + 1] = a1;
        }
    }
}

// ---- bound-ordered rerank ---------------------------------------------------------------------
//
// Per entry and mask, the set voxels of every 16 x 16 x 16 block of the grid (uint16
// [2][nbp], blocks (bz, by, bx) at (bz nby + by) nbx + bx, the rest zero). For a query with
// block counts a_b and a candidate with b_b, |A n B| <= sum over blocks of min(a_b, b_b), and
// Dice is increasing in |A n B|: the candidate's score is at most the same formula at those
// sums (in floating point too: the same operations on larger arguments). Scoring candidates
// in decreasing bound and leaving out those whose bound is below the k-th best exact score
// found gives the top k of scoring them all, bit for bit.

// Set voxels per block of the rows inside [z0, z1) x [y0, y1) of the two planes at P, into
// the LDS counts c[2][nbp] (zeroed before). With nxw % 4 == 0 an item is 16 bytes of a row
// (eight 16-voxel blocks), four items per thread in flight.
__device__ __forceinline__ void block_counts_rows(const uint32_t *__restrict__ P, int Wp, int nxw,
                                                  int ny, int z0, int z1, int y0, int y1, int nbx,
                                                  int nby, int nbp, uint32_t *c)
{
    const int nyr = y1 - y0;
    if (z1 <= z0 || nyr <= 0) return;
    const int rows = (z1 - z0) * nyr;
    if (nxw % 4 == 0) {
        // An item is 16 bytes (eight blocks) of the rows y of one 16-row block row at one
        // (plane, z): summed in registers, then one LDS add per block.
        const int nv = nxw / 4, yb0 = y0 >> 4, nyb = ((y1 - 1) >> 4) - yb0 + 1;
        const int items = 2 * (z1 - z0) * nyb * nv;
        for (int it = threadIdx.x; it < items; it += blockDim.x) {
            const int vi = it % nv, r1 = it / nv, yb = yb0 + r1 % nyb, r2 = r1 / nyb;
            const int pl = r2 & 1, z = z0 + (r2 >> 1);
            const int ya = max(y0, 16 * yb), yz = min(y1, 16 * yb + 16);
            const u32x4 *row = reinterpret_cast<const u32x4 *>(
                P + (int64_t)pl * Wp + ((int64_t)z * ny + ya) * nxw + 4 * vi);
            uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            for (int y = ya; y < yz; y += 4) {
                u32x4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    v[u] = y + u < yz ? row[(int64_t)(y - ya + u) * nv] : (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        acc[2 * t] += popc(v[u][t] & 0xffffu);
                        acc[2 * t + 1] += popc(v[u][t] >> 16);
                    }
            }
            const int at = pl * nbp + ((z >> 4) * nby + yb) * nbx + 8 * vi;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (acc[t]) atomicAdd(&c[at + t], acc[t]);
        }
        return;
    }
    const int items = rows * 2 * nxw;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int w = it % nxw, rem = it / nxw, pl = rem & 1, r = rem >> 1;
        const int z = z0 + r / nyr, y = y0 + r % nyr;
        const uint32_t word = P[(int64_t)pl * Wp + ((int64_t)z * ny + y) * nxw + w];
        if (word) {
            const int b = pl * nbp + ((z >> 4) * nby + (y >> 4)) * nbx + 2 * w;
            const uint32_t lo = popc(word & 0xffffu), hi = popc(word >> 16);
            if (lo) atomicAdd(&c[b], lo);
            if (hi) atomicAdd(&c[b + 1], hi);
        }
    }
}

// grid n entries, 256 threads: the block counts of entries e0 + blockIdx.x from their planes,
// inside their row boxes (zero outside).
__global__ void __launch_bounds__(256) block_count_kernel(const uint32_t *__restrict__ planes,
                                                          int Wp, int nxw, int ny,
                                                          const int32_t *__restrict__ box,
                                                          int nbx, int nby, int nbp,
                                                          uint16_t *__restrict__ bcnt)
{
    __shared__ uint32_t c[2 * kBoundMaxBlocks];
    const int64_t e = blockIdx.x;
    for (int i = threadIdx.x; i < 2 * nbp; i += blockDim.x) c[i] = 0u;
    __syncthreads();
    const int32_t *b = box + 4 * e;
    block_counts_rows(planes + e * 2 * Wp, Wp, nxw, ny, b[0], b[1], b[2], b[3], nbx, nby, nbp, c);
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * nbp; i += blockDim.x) bcnt[e * 2 * nbp + i] = (uint16_t)c[i];
}

// grid nq, 256 threads: the query's block counts (from its packed planes inside its row box)
// into qbc [nq][2][nbp] (uint32).
__global__ void __launch_bounds__(256) query_block_kernel(const uint32_t *__restrict__ qpack,
                                                          int Wp, int nxw, int ny,
                                                          const int32_t *__restrict__ box,
                                                          int nbx, int nby, int nbp,
                                                          uint32_t *__restrict__ qbc)
{
    __shared__ uint32_t c[2 * kBoundMaxBlocks];
    const int q = blockIdx.x;
    for (int i = threadIdx.x; i < 2 * nbp; i += blockDim.x) c[i] = 0u;
    __syncthreads();
    const int32_t *b = box + 4 * q;
    block_counts_rows(qpack + (int64_t)q * 2 * Wp, Wp, nxw, ny, b[0], b[1], b[2], b[3], nbx, nby,
                      nbp, c);
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * nbp; i += blockDim.x) qbc[(int64_t)q * 2 * nbp + i] = c[i];
}

// One wave per four candidates of a query (blocks of four waves): each candidate's bound into
// ub [nq][nc], the loads of the four issued together. With nbx % 8 == 0 a 16-byte chunk of
// counts is eight blocks of one (bz, by) block row, and only the block rows the query's row
// box meets are read (the query's counts are zero elsewhere).
__global__ void __launch_bounds__(256) rerank_ub_kernel(const uint16_t *__restrict__ bcnt,
                                                        int nbx, int nby, int nbp,
                                                        const uint32_t *__restrict__ popcnt,
                                                        const uint32_t *__restrict__ qbc,
                                                        const int32_t *__restrict__ box,
                                                        const uint32_t *__restrict__ acnt,
                                                        const int32_t *__restrict__ cand, int nc,
                                                        int nq, double *__restrict__ ub)
{
    constexpr int C = 4, CH = 2;               // candidates per wave; chunks per lane and pass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = (nc + 4 * C - 1) / (4 * C);
    const int q = blockIdx.x / per, c0 = ((blockIdx.x % per) * 4 + wave) * C;
    if (q >= nq || c0 >= nc) return;           // a whole wave leaves; no block barrier below
    const int64_t qo = (int64_t)q * nc;
    const int32_t *b = box + 4 * q;
    const bool rows = nbx % 8 == 0;
    const int bz0 = b[0] >> 4, bz1 = b[1] > b[0] ? (b[1] - 1) >> 4 : -1;
    const int by0 = b[2] >> 4, by1 = b[3] > b[2] ? (b[3] - 1) >> 4 : -1;
    const uint32_t *Q = qbc + (int64_t)q * 2 * nbp;
    const int nch = nbp / 8;                   // 16-byte chunks per plane
    int32_t e[C];
#pragma unroll
    for (int j = 0; j < C; ++j) e[j] = cand[qo + min(c0 + j, nc - 1)];
    uint32_t u0[C] = {}, u1[C] = {};
    for (int ch0 = lane; ch0 < 2 * nch; ch0 += 64 * CH) {
        bool use[CH];
        u32x4 v[CH][C];
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            const int ch = ch0 + 64 * h;
            const int pl = ch >= nch, b0 = 8 * (ch - pl * nch);
            bool in = ch < 2 * nch;
            if (rows && in) {
                const int br = b0 / nbx, bz = br / nby, by = br - bz * nby;
                in = bz >= bz0 && bz <= bz1 && by >= by0 && by <= by1;   // padding: bz >= nbz
            }
            use[h] = in;
#pragma unroll
            for (int j = 0; j < C; ++j)
                v[h][j] = in ? reinterpret_cast<const u32x4 *>(bcnt + (int64_t)e[j] * 2 * nbp)[ch]
                             : (u32x4){0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            if (!use[h]) continue;
            const int ch = ch0 + 64 * h;
            const u32x4 qa = *reinterpret_cast<const u32x4 *>(Q + 8 * ch);    // 32-byte aligned
            const u32x4 qb = *reinterpret_cast<const u32x4 *>(Q + 8 * ch + 4);
            const uint32_t qv[8] = {qa[0], qa[1], qa[2], qa[3], qb[0], qb[1], qb[2], qb[3]};
#pragma unroll
            for (int j = 0; j < C; ++j) {
                uint32_t m = 0u;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    m += min(v[h][j][t] & 0xffffu, qv[2 * t]) + min(v[h][j][t] >> 16, qv[2 * t + 1]);
                if (ch >= nch) u1[j] += m;
                else u0[j] += m;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const uint32_t a0 = wave_sum(u0[j]), a1 = wave_sum(u1[j]);
        if (lane == 0 && c0 + j < nc)
            ub[qo + c0 + j] = dice(a1, acnt[2 * q + 1], popcnt[2 * (int64_t)e[j] + 1]) +
                              dice(a0, acnt[2 * q], popcnt[2 * (int64_t)e[j]]);
    }
}

// grid nq, 256 threads: the query's candidates sorted by (bound desc, slot asc) into order /
// ubs [nq][nc]; every slot's score set to the smallest positive double's bits (below any
// score a ranked candidate can have once it is left out) and its entry index.
__global__ void __launch_bounds__(256) rerank_order_kernel(const double *__restrict__ ub,
                                                           const int32_t *__restrict__ cand, int nc,
                                                           int32_t *__restrict__ order,
                                                           double *__restrict__ ubs,
                                                           int32_t *__restrict__ ents,
                                                           uint64_t *__restrict__ ws_s,
                                                           int32_t *__restrict__ ws_i)
{
    __shared__ double sk[kRerankMaxCand];
    __shared__ int32_t si[kRerankMaxCand];
    const int64_t qo = (int64_t)blockIdx.x * nc;
    int P = 1;
    while (P < nc) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        sk[t] = t < nc ? ub[qo + t] : -1.0;
        si[t] = t < nc ? t : INT_MAX;
        if (t < nc) {
            ws_s[qo + t] = 1ull;
            ws_i[qo + t] = cand[qo + t];
        }
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const double ki = sk[i], kj = sk[j];
                const int32_t ii = si[i], ij = si[j];
                const bool j_first = kj > ki || (kj == ki && ij < ii);
                if (j_first == up) {
                    sk[i] = kj;
                    sk[j] = ki;
                    si[i] = ij;
                    si[j] = ii;
                }
            }
        }
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
        order[qo + t] = si[t];
        ubs[qo + t] = sk[t];
        ents[qo + t] = cand[qo + si[t]];
    }
}

// One wave per query (grid ceil(nq / 4), 256 threads), after the first n1 positions in bound
// order are scored: tau = the k-th best of their scores (k <= n1 <= 64), and qcount[q] = the
// positions from n1 on whose bound reaches tau (a prefix: the bounds are sorted). Every other
// candidate's score is at most its bound < tau, below the k best.
__global__ void __launch_bounds__(256) rerank_gate_kernel(const uint64_t *__restrict__ ws_s,
                                                          const int32_t *__restrict__ order,
                                                          const double *__restrict__ ubs, int nc,
                                                          int n1, int k, int nq,
                                                          int32_t *__restrict__ qcount)
{
    const int lane = threadIdx.x & 63, q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    const int64_t qo = (int64_t)q * nc;
    const double v = lane < n1 ? __longlong_as_double((long long)ws_s[qo + order[qo + lane]])
                               : -INFINITY;
    int rank = 0;
    for (int l = 0; l < n1; ++l) {
        const double w = __shfl(v, l);
        rank += (w > v || (w == v && l < lane)) ? 1 : 0;
    }
    const uint64_t hit = __ballot(lane < n1 && rank == k - 1);
    const double tau = __shfl(v, (int)__builtin_ctzll(hit));
    int n2 = 0;
    for (int i0 = n1; i0 < nc; i0 += 64) {
        const int i = i0 + lane;
        const uint64_t in = __ballot(i < nc && ubs[qo + i] >= tau);
        n2 += __builtin_popcountll(in);
        if (in != __ballot(i < nc)) break;     // the prefix ended in this pass
    }
    if (lane == 0) qcount[q] = n2;
}

// grid nq, 256 threads: rank the query's nc scored candidates by (score desc,
// index asc) in LDS (bitonic over slot numbers) and write the first k.
__global__ void __launch_bounds__(256) rerank_rank_kernel(const uint32_t *__restrict__ popcnt,
                                                          const uint32_t *__restrict__ acnt, int nc,
                                                          int k, const uint64_t *__restrict__ ws_s,
                                                          const int32_t *__restrict__ ws_i,
                                                          const uint32_t *__restrict__ ws_I,
                                                          int32_t *__restrict__ out_idx,
                                                          double *__restrict__ out_score,
                                                          db_counts_t *__restrict__ out_counts)
{
    __shared__ uint64_t ks[kRerankMaxCand];
    __shared__ int32_t ki[kRerankMaxCand];
    __shared__ int16_t slot[kRerankMaxCand];
    const int q = blockIdx.x;
    int P = 1;
    while (P < nc) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const bool in = t < nc;
        ks[t] = in ? ws_s[(int64_t)q * nc + t] : 0ull;
        ki[t] = in ? ws_i[(int64_t)q * nc + t] : INT_MAX;
        slot[t] = (int16_t)t;
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const int si_ = slot[i], sj = slot[j];
                if (ranks_before(ks[sj], ki[sj], ks[si_], ki[si_]) == up) {
                    slot[i] = (int16_t)sj;
                    slot[j] = (int16_t)si_;
                }
            }
        }
    __syncthreads();
    const uint32_t A0 = acnt[2 * q], A1 = acnt[2 * q + 1];
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        const int sl = slot[t];
        const int64_t o = (int64_t)q * k + t;
        const int32_t e = ki[sl];
        out_idx[o] = e;
        out_score[o] = __longlong_as_double((long long)ks[sl]);
        if (out_counts) {
            db_counts_t cc;
            cc.inter[0] = ws_I[2 * ((int64_t)q * nc + sl)];
            cc.inter[1] = ws_I[2 * ((int64_t)q * nc + sl) + 1];
            cc.a[0] = A0;
            cc.a[1] = A1;
            cc.b[0] = popcnt[2 * (int64_t)e];
            cc.b[1] = popcnt[2 * (int64_t)e + 1];
            out_counts[o] = cc;
        }
    }
}

// ---- two-stage exact k smallest: per chunk, then a merge ------------------------------------

constexpr int kChunkThreads = 512;
constexpr int kChunkPer = 24;                          // keys per thread, held in registers
constexpr int kChunk = kChunkThreads * kChunkPer;      // 12,288 row entries per block
constexpr int kChunkWaves = kChunkThreads / 64;
constexpr int kMergeMax = 8192;                        // candidates per row the merge sorts

// grid (chunks, M), kChunkThreads threads; entry base + u * kChunkThreads + tid
// of the row is key u of thread tid. The key T of the chunk's k-th smallest
// entry is found by bisection on the key range [min, max]: the smallest T
// with at least k keys <= T (at most 32 block-wide counts, no histograms).
// The block writes its k smallest (key, index) pairs, ties at T by lowest
// index, unsorted (a chunk shorter than k writes all of its entries and pads
// with (max key, INT_MAX)). The union of the chunks' k smallest holds the
// row's k smallest under the (key, index) order.
__global__ void __launch_bounds__(kChunkThreads) topk_chunk_kernel(const float *__restrict__ D,
                                                                   int N, int k,
                                                                   uint32_t *__restrict__ ck,
                                                                   int32_t *__restrict__ ci)
{
    __shared__ uint32_t red[3][kChunkWaves];
    __shared__ uint32_t wcnt[kChunkPer * kChunkWaves];
    __shared__ uint32_t scan[256];
    __shared__ uint32_t s_lt;
    static_assert(kChunkPer * kChunkWaves <= 256, "scan size");
    const int c = blockIdx.x, nch = gridDim.x;
    const int base = c * kChunk;
    const int len = min(kChunk, N - base);
    const float *row = D + (int64_t)blockIdx.y * N + base;
    uint32_t *okey = ck + ((int64_t)blockIdx.y * nch + c) * k;
    int32_t *oidx = ci + ((int64_t)blockIdx.y * nch + c) * k;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t key[kChunkPer];
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int i = u * kChunkThreads + tid;
        key[u] = i < len ? fkey(row[i]) : 0u;
    }
    auto valid = [&](int u) { return u * kChunkThreads + tid < len; };
    if (len <= k) {
#pragma unroll
        for (int u = 0; u < kChunkPer; ++u) {
            const int i = u * kChunkThreads + tid;
            if (i < k) {
                okey[i] = i < len ? key[u] : 0xffffffffu;
                oidx[i] = i < len ? base + i : INT_MAX;
            }
        }
        return;                          // k <= DB_KMAX < kChunk: every slot was written
    }
    // Key range of the chunk.
    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u)
        if (valid(u)) {
            lo = min(lo, key[u]);
            hi = max(hi, key[u]);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
    }
    if (lane == 0) {
        red[0][wave] = lo;
        red[1][wave] = hi;
    }
    __syncthreads();
    lo = red[0][0];
    hi = red[1][0];
    for (int w = 1; w < kChunkWaves; ++w) {
        lo = min(lo, red[0][w]);
        hi = max(hi, red[1][w]);
    }
    __syncthreads();
    // Bisection: smallest T in [lo, hi] with count(key <= T) >= k. Each round's
    // block-wide count goes through red[round % 3]: a slot is cleared two rounds
    // before its next use, after every thread has read it.
    const uint32_t kk = (uint32_t)k;
    uint32_t below = 0;                 // count(key <= lo - 1) once lo has moved
    int round = 0;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        uint32_t cnt = 0;
#pragma unroll
        for (int u = 0; u < kChunkPer; ++u) cnt += (valid(u) && key[u] <= mid) ? 1u : 0u;
        cnt = wave_sum(cnt);
        const int slot = round % 3;
        if (lane == 0) red[slot][wave] = cnt;
        __syncthreads();
        uint32_t total = 0;
        for (int w = 0; w < kChunkWaves; ++w) total += red[slot][w];
        if (total >= kk) {
            hi = mid;
        } else {
            lo = mid + 1;
            below = total;
        }
        ++round;
    }
    const uint32_t T = lo;
    const uint32_t remaining = kk - below;
    // Keys below T: any order. Keys equal to T: the first `remaining` by index.
    uint32_t eq = 0;
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) eq += (valid(u) && key[u] == T) ? 1u : 0u;
    eq = wave_sum(eq);
    if (tid == 0) s_lt = 0;
    __syncthreads();
    if (lane == 0) atomicAdd(&s_lt, eq);   // s_lt temporarily holds count(key == T)
    __syncthreads();
    const bool all_eq = s_lt == remaining;
    __syncthreads();
    if (tid == 0) s_lt = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const int i = u * kChunkThreads + tid;
        if (valid(u) && (key[u] < T || (all_eq && key[u] == T))) {
            const uint32_t slot = atomicAdd(&s_lt, 1u);
            okey[slot] = key[u];
            oidx[slot] = base + i;
        }
    }
    if (all_eq) return;
    // Ordered pick among the keys equal to T: per (register, wave) counts in
    // index order, an exclusive scan, then each lane's rank.
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const uint64_t bm = __ballot(valid(u) && key[u] == T);
        if (lane == 0) wcnt[u * kChunkWaves + wave] = (uint32_t)__popcll(bm);
    }
    __syncthreads();
    {   // exclusive scan of the kChunkPer * kChunkWaves (<= 256) counts
        constexpr int n = kChunkPer * kChunkWaves;
        const uint32_t v = tid < n ? wcnt[tid] : 0u;
        if (tid < 256) scan[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const uint32_t y = (tid < 256 && tid >= off) ? scan[tid - off] : 0u;
            __syncthreads();
            if (tid < 256) scan[tid] += y;
            __syncthreads();
        }
        if (tid < n) wcnt[tid] = scan[tid] - v;
        __syncthreads();
    }
    const uint32_t n_lt = kk - remaining;
    const uint64_t lower = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int u = 0; u < kChunkPer; ++u) {
        const bool p = valid(u) && key[u] == T;
        const uint64_t bm = __ballot(p);
        if (p) {
            const uint32_t r = wcnt[u * kChunkWaves + wave] + (uint32_t)__popcll(bm & lower);
            if (r < remaining) {
                okey[n_lt + r] = T;
                oidx[n_lt + r] = base + u * kChunkThreads + tid;
            }
        }
    }
}

// grid M, kSelThreads threads: sort the row's nc <= kMergeMax candidates by
// (key, index) in LDS (bitonic) and write the first k.
__global__ void __launch_bounds__(kSelThreads) topk_merge_kernel(int nc, int k,
                                                                 const uint32_t *__restrict__ ck,
                                                                 const int32_t *__restrict__ ci,
                                                                 int32_t *__restrict__ out_idx,
                                                                 float *__restrict__ out_d)
{
    __shared__ uint32_t sk[kMergeMax];
    __shared__ int32_t si[kMergeMax];
    const int64_t r = blockIdx.x;
    int P = 1;
    while (P < nc) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        sk[t] = t < nc ? ck[r * nc + t] : 0xffffffffu;
        si[t] = t < nc ? ci[r * nc + t] : INT_MAX;
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint32_t ki = sk[i], kj = sk[j];
                const int32_t ii = si[i], ij = si[j];
                const bool j_first = kj < ki || (kj == ki && ij < ii);
                if (j_first == up) {
                    sk[i] = kj;
                    sk[j] = ki;
                    si[i] = ij;
                    si[j] = ii;
                }
            }
        }
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        out_idx[r * k + t] = si[t];
        out_d[r * k + t] = fkey_inv(sk[t]);
    }
}

// ---- k smallest by a bound and a filter (long rows, small k) -------------------------------
//
// For a row of N entries cut into C full chunks of kTauChunk, let tau_c be the
// m-th smallest of the chunk's per-thread minima (m = ceil(k / C)). At least m
// entries of chunk c are <= tau_c, so at least C * m >= k entries of the row
// are <= tau = max_c tau_c: the row's k smallest are all <= tau. One streaming
// pass finds tau (an atomic max per chunk) and keeps every thread's minimum; a
// block per row then reads only the entries of threads whose minimum is <= tau
// (a few hundred entries per row at the workloads here), and sorts them by
// (key, index). A row with more than kTauCap such entries is selected by the
// one-block radix path instead.

constexpr int kTauThreads = 512;
constexpr int kTauMaxM = 8;     // m <= 8: the 8 waves' 8 smallest minima fill one wave
constexpr int kTauCap = 4096;
// Entries per thread: 16 (chunks of 8,192) for long rows, 4 (chunks of 2,048) where
// that gives too few chunks for m <= kTauMaxM.

// Minimum of v over the wave (all lanes active), the same in every lane: DPP
// rotations within each row of 16, then the four row results.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    v = min(v, dpp_u32<0x128>(v));   // row_ror 8
    v = min(v, dpp_u32<0x124>(v));   // row_ror 4
    v = min(v, dpp_u32<0x122>(v));   // row_ror 2
    v = min(v, dpp_u32<0x121>(v));   // row_ror 1
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(a, b), min(c, d));
}

// The m smallest of the wave's values v (one per lane; m <= kTauMaxM), ascending, into
// out[0..m) (written by lane 0): m rounds of a wave minimum, each removing one lane
// holding it (the lowest), so equal values count once per lane.
__device__ __forceinline__ void wave_smallest(uint32_t v, int m, int lane, uint32_t *out)
{
    for (int i = 0; i < m; ++i) {
        const uint32_t mn = wave_min_u32(v);
        const uint64_t hold = __ballot(v == mn);
        if (lane == __ffsll((unsigned long long)hold) - 1) v = 0xffffffffu;
        if (lane == 0) out[i] = mn;
    }
}

// m-th smallest (1 <= m <= kTauMaxM) of one value per thread of a block of W waves:
// each wave's m smallest into wl, then the m smallest of those W * m in wave 0. The
// result is valid in wave 0 (returned there; other waves return 0).
template <int W>
__device__ __forceinline__ uint32_t block_mth_smallest(uint32_t v, int m, uint32_t (&wl)[W][kTauMaxM])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    wave_smallest(v, m, lane, wl[wave]);
    __syncthreads();
    if (wave != 0) return 0;
    uint32_t x = lane < W * m ? wl[lane / m][lane % m] : 0xffffffffu;
    uint32_t mth = 0;
    for (int i = 0; i < m; ++i) {
        mth = wave_min_u32(x);
        const uint64_t hold = __ballot(x == mth);
        if (lane == __ffsll((unsigned long long)hold) - 1) x = 0xffffffffu;
    }
    return mth;
}

// grid (C, M), kTauThreads threads: tau[row] = max(tau[row], m-th smallest thread minimum);
// each thread's minimum is kept in tmin [M][C][kTauThreads] for the filter pass.
template <int kTauPer>
__global__ void __launch_bounds__(kTauThreads) topk_tau_kernel(const float *__restrict__ D, int N,
                                                               int m, uint32_t *__restrict__ tau,
                                                               uint32_t *__restrict__ tmin)
{
    constexpr int kTauChunk = kTauThreads * kTauPer;
    __shared__ uint32_t wl[kTauThreads / 64][kTauMaxM];
    const int64_t r = blockIdx.y;
    const int base = blockIdx.x * kTauChunk;
    if (N - base < kTauChunk) return;                 // partial chunk: no bound from it
    const float *row = D + r * N + base;
    const int tid = threadIdx.x;
    uint32_t mn = 0xffffffffu;
    if ((N & 3) == 0) {      // 16-byte aligned rows: 4 entries per load
        const f32x4 *row4 = reinterpret_cast<const f32x4 *>(row);
#pragma unroll
        for (int u = 0; u < kTauPer / 4; ++u) {
            const f32x4 x = __builtin_nontemporal_load(row4 + u * kTauThreads + tid);
#pragma unroll
            for (int e = 0; e < 4; ++e) mn = min(mn, fkey(x[e]));
        }
    } else {
#pragma unroll
        for (int u = 0; u < kTauPer; ++u) mn = min(mn, fkey(row[u * kTauThreads + tid]));
    }
    tmin[((int64_t)r * gridDim.x + blockIdx.x) * kTauThreads + tid] = mn;
    const uint32_t mth = block_mth_smallest<kTauThreads / 64>(mn, m, wl);
    if (tid == 0) atomicMax(&tau[r], mth);
}

// The list of nc (key, index) pairs in LDS (the block's gather, after a barrier):
// sort by (key, index) and write the first k. A list longer than kTauCap was not
// kept whole: the row is selected by the one-block radix path instead.
__device__ __forceinline__ void list_sort_emit(uint32_t *sk, int32_t *si, uint32_t nc,
                                               const float *__restrict__ row, int N, int k,
                                               int32_t *__restrict__ out_idx,
                                               float *__restrict__ out_d)
{
    if (nc > (uint32_t)kTauCap) {
        select_row_radix(row, N, k, out_idx, out_d);
        return;
    }
    int P = 1;
    while (P < (int)nc) P <<= 1;
    for (int q = (int)nc + threadIdx.x; q < P; q += blockDim.x) {
        sk[q] = 0xffffffffu;
        si[q] = INT_MAX;
    }
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int q = threadIdx.x; q < P / 2; q += blockDim.x) {
                const int i = 2 * q - (q & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint32_t ki = sk[i], kj = sk[j];
                const int32_t ii = si[i], ij = si[j];
                const bool j_first = kj < ki || (kj == ki && ij < ii);
                if (j_first == up) {
                    sk[i] = kj;
                    sk[j] = ki;
                    si[i] = ij;
                    si[j] = ii;
                }
            }
        }
    __syncthreads();
    for (int q = threadIdx.x; q < k; q += blockDim.x) {
        out_idx[q] = si[q];
        out_d[q] = fkey_inv(sk[q]);
    }
}

// grid M, kSelThreads threads: gather the row's entries with key <= tau[row] into
// LDS (in a full chunk only the threads whose minimum is <= tau hold any: their
// 16 entries are read; the partial last chunk is read whole), sort them by
// (key, index) and write the first k. A list longer than kTauCap falls back to
// the one-block radix selection of the whole row.
template <int kTauPer>
__global__ void __launch_bounds__(kSelThreads) topk_list_kernel(const float *__restrict__ D, int N,
                                                                int k, const uint32_t *__restrict__ tau,
                                                                const uint32_t *__restrict__ tmin,
                                                                int32_t *__restrict__ out_idx,
                                                                float *__restrict__ out_d)
{
    constexpr int kTauChunk = kTauThreads * kTauPer;
    __shared__ uint32_t sk[kTauCap];
    __shared__ int32_t si[kTauCap];
    __shared__ uint32_t s_n;
    const int64_t r = blockIdx.x;
    const float *row = D + r * N;
    const uint32_t t = tau[r];
    const int cfull = N / kTauChunk;
    const int slots = cfull * kTauThreads;
    const bool v4 = (N & 3) == 0;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    auto push = [&](uint32_t key, int i) {
        const uint32_t pos = atomicAdd(&s_n, 1u);
        if (pos < (uint32_t)kTauCap) {
            sk[pos] = key;
            si[pos] = i;
        }
    };
    for (int sl = threadIdx.x; sl < slots; sl += blockDim.x) {
        if (tmin[r * slots + sl] > t) continue;
        const int c = sl / kTauThreads, th = sl - c * kTauThreads;
        const int base = c * kTauChunk;
        if (v4) {
            const f32x4 *row4 = reinterpret_cast<const f32x4 *>(row + base);
#pragma unroll
            for (int u = 0; u < kTauPer / 4; ++u) {
                const int j = u * kTauThreads + th;
                const f32x4 x = row4[j];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t key = fkey(x[e]);
                    if (key <= t) push(key, base + 4 * j + e);
                }
            }
        } else {
#pragma unroll 4
            for (int u = 0; u < kTauPer; ++u) {
                const int i = base + u * kTauThreads + th;
                const uint32_t key = fkey(row[i]);
                if (key <= t) push(key, i);
            }
        }
    }
    for (int i = cfull * kTauChunk + threadIdx.x; i < N; i += blockDim.x) {
        const uint32_t key = fkey(row[i]);
        if (key <= t) push(key, i);
    }
    __syncthreads();
    list_sort_emit(sk, si, s_n, row, N, k, out_idx + r * k, out_d + r * k);
}

// ---- the same bound from the distance kernel's group minima ------------------------------
//
// With GMIN the distance kernel leaves, per row, the minimum key of every whole
// group of 16 consecutive entries. A chunk of CG groups (CG * 16 entries) has
// at least m entries <= the m-th smallest of its group minima, so the bound
// above holds with groups in place of threads, and it is found by reading
// 1/16 of the distances' bytes; the gather reads only the groups whose minimum
// is <= tau (and the entries after the last whole chunk).

// grid (ceil(C / (4 CPW)), M), 256 threads: wave w of block x takes chunks
// CPW (4x + w) .. + CPW - 1 (those < C) of 64 * PER group minima each, PER per lane,
// all loaded before any is used; for each it finds the m-th smallest (m rounds of a
// wave minimum over the lanes' smallest remaining values, each round removing one
// copy of it) and raises tau[row] to the largest of those.
template <int PER, int CPW>
__global__ void __launch_bounds__(256) topk_tau_groups_kernel(const uint32_t *__restrict__ gmin,
                                                             int64_t gld, int chunks, int m,
                                                             uint32_t *__restrict__ tau)
{
    const int lane = threadIdx.x & 63;
    const int c0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * CPW;
    if (c0 >= chunks) return;                     // whole wave; no barriers here
    const int nc = min(CPW, chunks - c0);
    const int64_t r = blockIdx.y;
    const uint32_t *p = gmin + r * gld + (int64_t)c0 * 64 * PER;
    uint32_t v[CPW][PER];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int q = 0; q < PER; ++q) v[c][q] = c < nc ? p[(c * PER + q) * 64 + lane] : 0u;
    uint32_t best = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        if (c >= nc) break;                       // uniform over the wave
        auto lane_min = [&]() {
            uint32_t x = v[c][0];
#pragma unroll
            for (int q = 1; q < PER; ++q) x = min(x, v[c][q]);
            return x;
        };
        uint32_t lm = lane_min(), mn = 0;
        for (int i = 0;; ++i) {
            mn = wave_min_u32(lm);
            if (i + 1 == m) break;
            const uint64_t hold = __ballot(lm == mn);
            if (lane == __ffsll((unsigned long long)hold) - 1) {
                bool done = false;
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    if (!done && v[c][q] == mn) {
                        v[c][q] = 0xffffffffu;
                        done = true;
                    }
                lm = lane_min();
            }
        }
        best = max(best, mn);
    }
    if (lane == 0) atomicMax(&tau[r], best);
}

// grid M, kSelThreads threads: the entries of row r with key <= tau[r], from the
// groups g < nslots whose minimum is <= tau and from entries nslots * 16 .. N - 1;
// sorted, the first k written.
__global__ void __launch_bounds__(kSelThreads) topk_list_groups_kernel(
    const float *__restrict__ D, int N, int k, const uint32_t *__restrict__ tau,
    const uint32_t *__restrict__ gmin, int64_t gld, int nslots, int32_t *__restrict__ out_idx,
    float *__restrict__ out_d)
{
    __shared__ uint32_t sk[kTauCap];
    __shared__ int32_t si[kTauCap];
    __shared__ uint32_t s_n;
    const int64_t r = blockIdx.x;
    const float *row = D + r * N;
    const uint32_t t = tau[r];
    const bool v4 = (N & 3) == 0;                 // 16-byte aligned rows
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    auto push = [&](uint32_t key, int i) {
        const uint32_t pos = atomicAdd(&s_n, 1u);
        if (pos < (uint32_t)kTauCap) {
            sk[pos] = key;
            si[pos] = i;
        }
    };
    auto gather = [&](int g) {                    // the 16 entries of group g
        const int base = 16 * g;
        if (v4) {
            const f32x4 *p = reinterpret_cast<const f32x4 *>(row + base);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 x = p[q];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t key = fkey(x[e]);
                    if (key <= t) push(key, base + 4 * q + e);
                }
            }
        } else {
#pragma unroll 4
            for (int e = 0; e < 16; ++e) {
                const uint32_t key = fkey(row[base + e]);
                if (key <= t) push(key, base + e);
            }
        }
    };
    // Four group minima in flight per thread, then the groups that pass.
    for (int g0 = threadIdx.x; g0 < nslots; g0 += 4 * kSelThreads) {
        uint32_t gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int g = g0 + u * kSelThreads;
            gv[u] = g < nslots ? gmin[r * gld + g] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (gv[u] <= t) gather(g0 + u * kSelThreads);
    }
    for (int i = 16 * nslots + threadIdx.x; i < N; i += blockDim.x) {
        const uint32_t key = fkey(row[i]);
        if (key <= t) push(key, i);
    }
    __syncthreads();
    list_sort_emit(sk, si, s_n, row, N, k, out_idx + r * k, out_d + r * k);
}

// Groups per chunk for (N, k): 512 (8,192 entries) for long rows, else 128 (2,048),
// whichever gives m = ceil(k / full chunks) <= kTauMaxM; 0 when neither does.
static int groups_cg(int N, int k)
{
    for (int cg : {512, 128}) {
        const int full = N / (cg * 16);
        if (full >= 1 && (k + full - 1) / full <= kTauMaxM) return cg;
    }
    return 0;
}

size_t topk_groups_ws_bytes(int M, int N)
{
    return align_up((size_t)M * 4, kAlign) + (size_t)M * (N / 16) * 4;
}

uint32_t *topk_groups_gmin(void *ws, int M)
{
    return reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + align_up((size_t)M * 4, kAlign));
}

hipError_t launch_topk_groups(int M, int N, int k, const float *D, void *ws, int32_t *idx,
                              float *d, hipStream_t s)
{
    const int cg = groups_cg(N, k);
    if (cg == 0) {                                 // no bound: one block per row
        hipLaunchKernelGGL(topk_min_kernel, dim3(M), dim3(kSelThreads), 0, s, D, N, k, idx, d);
        return hipGetLastError();
    }
    const int full = N / (cg * 16), m = (k + full - 1) / full;
    uint32_t *tau = static_cast<uint32_t *>(ws);
    const uint32_t *gmin = topk_groups_gmin(ws, M);
    const int64_t gld = N / 16;
    hipError_t e = launch_fill_u32(reinterpret_cast<int32_t *>(tau), M, 0, s);
    if (e != hipSuccess) return e;
    constexpr int kCpw = 4;                        // chunks per wave
    const unsigned bx = (unsigned)((full + 4 * kCpw - 1) / (4 * kCpw));
    if (cg == 512)
        hipLaunchKernelGGL((topk_tau_groups_kernel<8, kCpw>), dim3(bx, M), dim3(256), 0, s, gmin, gld,
                           full, m, tau);
    else
        hipLaunchKernelGGL((topk_tau_groups_kernel<2, kCpw>), dim3(bx, M), dim3(256), 0, s, gmin, gld,
                           full, m, tau);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(topk_list_groups_kernel, dim3(M), dim3(kSelThreads), 0, s, D, N, k, tau, gmin,
                       gld, full * cg, idx, d);
    return hipGetLastError();
}

// ---- launchers ---------------------------------------------------------------------------------

hipError_t launch_quant_bf16(int64_t n, int dim, const float *x, uint16_t *y, float *sq,
                             hipStream_t s)
{
    hipLaunchKernelGGL(quant_bf16_kernel, dim3((unsigned)n), dim3(256), 0, s, dim, x, y, sq);
    return hipGetLastError();
}

hipError_t launch_quant_fp8(int64_t n, int dim, const float *x, uint8_t *y, float *scale,
                            float *sq, hipStream_t s)
{
    hipLaunchKernelGGL(quant_fp8_kernel, dim3((unsigned)n), dim3(256), 0, s, dim, x, y, scale, sq);
    return hipGetLastError();
}

// Persistent grid of the distance kernel: as many blocks as fit on the device
// at once (a multiple of 8, so each block keeps its XCD), at most one per tile.
// X is taken in chunks of fewer than 2^31 bytes (32-bit row offsets), each
// chunk one launch writing its columns of D (and its groups of gmin).
template <bool FP8, bool TAIL, int DEPTH, bool GMIN>
static hipError_t dist_lds_launch(int M, int N, int K, const uint8_t *Q, const float *qs,
                                  const float *qn, const uint8_t *X, const float *xs,
                                  const float *xn, float *D, int mode, uint32_t *gmin,
                                  hipStream_t s)
{
    static int resident[64];                        // per device: blocks resident at once
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (resident[dev] == 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, dist_lds_kernel<FP8, TAIL, DEPTH, GMIN>, kDThreads, 0);
        if (e != hipSuccess) return e;
        resident[dev] = max(kXcds, (cus * max(per_cu, 1)) / kXcds * kXcds);
    }
    const int64_t Kb = FP8 ? K : 2 * (int64_t)K;
    if ((int64_t)M * Kb >= kDChunkBytes) return hipErrorInvalidValue;
    const int chunk = (int)(((kDChunkBytes - 1) / Kb) / kDN * kDN);   // a multiple of 16
    const int mt = (M + kDM - 1) / kDM;
    for (int c0 = 0; c0 < N; c0 += chunk) {
        const int n = min(chunk, N - c0);
        const int nt = (n + kDN - 1) / kDN;
        const int ntiles = kXcds * mt * ((nt + kXcds - 1) / kXcds);   // a multiple of 8
        const int g = min(ntiles, resident[dev]);
        hipLaunchKernelGGL((dist_lds_kernel<FP8, TAIL, DEPTH, GMIN>), dim3(g), dim3(kDThreads), 0, s,
                           M, n, K, mt, ntiles, Q, qs, qn, X + c0 * Kb, FP8 ? xs + c0 : nullptr,
                           xn + c0, D ? D + c0 : nullptr, (int64_t)N, mode, GMIN ? gmin + c0 / 16 : nullptr,
                           (int64_t)(N / 16), n / 16);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Register ring depth (K slices in flight per block): one, which keeps the kernel
// within 128 VGPRs (two blocks per CU) for both formats.
constexpr int kDDepthBf16 = 1, kDDepthFp8 = 1;

hipError_t launch_dist_bf16(int M, int N, int K, const uint16_t *Q, const float *qn,
                            const uint16_t *X, const float *xn, float *D, int mode,
                            uint32_t *gmin, hipStream_t s)
{
    const auto *q = reinterpret_cast<const uint8_t *>(Q);
    const auto *x = reinterpret_cast<const uint8_t *>(X);
    if (gmin) {
        if (mode != 0) return hipErrorInvalidValue;
        if ((2 * K) % kDSlice)
            return dist_lds_launch<false, true, kDDepthBf16, true>(M, N, K, q, nullptr, qn, x,
                                                                   nullptr, xn, D, 0, gmin, s);
        return dist_lds_launch<false, false, kDDepthBf16, true>(M, N, K, q, nullptr, qn, x,
                                                                nullptr, xn, D, 0, gmin, s);
    }
    if ((2 * K) % kDSlice)
        return dist_lds_launch<false, true, kDDepthBf16, false>(M, N, K, q, nullptr, qn, x, nullptr,
                                                                xn, D, mode, nullptr, s);
    return dist_lds_launch<false, false, kDDepthBf16, false>(M, N, K, q, nullptr, qn, x, nullptr,
                                                             xn, D, mode, nullptr, s);
}

hipError_t launch_dist_fp8(int M, int N, int K, const uint8_t *Q, const float *qs, const float *qn,
                           const uint8_t *X, const float *xs, const float *xn, float *D,
                           int mode, uint32_t *gmin, hipStream_t s)
{
    if (K % kDSlice) return hipErrorInvalidValue;   // FP8 rows are whole slices
    if (gmin) {
        if (mode != 0) return hipErrorInvalidValue;
        return dist_lds_launch<true, false, kDDepthFp8, true>(M, N, K, Q, qs, qn, X, xs, xn, D, 0,
                                                              gmin, s);
    }
    return dist_lds_launch<true, false, kDDepthFp8, false>(M, N, K, Q, qs, qn, X, xs, xn, D, mode,
                                                           nullptr, s);
}

// m of the bound-and-filter path with `per` entries per thread, or 0 when it does not
// apply (too few full chunks).
static int tau_m_per(int N, int k, int per)
{
    const int full = N / (kTauThreads * per);
    if (full < 1) return 0;
    const int m = (k + full - 1) / full;
    return m <= kTauMaxM ? m : 0;
}

// Entries per thread of the bound-and-filter path for (N, k): 16, else 4, else 0 (n/a).
static int tau_per(int N, int k)
{
    if (tau_m_per(N, k, 16)) return 16;
    if (tau_m_per(N, k, 4)) return 4;
    return 0;
}

size_t topk_min_ws_bytes(int M, int N, int k)
{
    if (const int per = tau_per(N, k))
        return align_up((size_t)M * 4, kAlign) +
               (size_t)M * (N / (kTauThreads * per)) * kTauThreads * 4;
    const int64_t nch = ((int64_t)N + kChunk - 1) / kChunk;
    if (nch * k > kMergeMax) return 0;       // the two-stage path does not apply
    return (size_t)M * nch * k * 8;
}

hipError_t launch_topk_min(int M, int N, int k, const float *D, int32_t *idx, float *d, void *ws,
                           size_t ws_bytes, hipStream_t s)
{
    const size_t need = topk_min_ws_bytes(M, N, k);
    if (!ws || need == 0 || ws_bytes < need) {
        hipLaunchKernelGGL(topk_min_kernel, dim3(M), dim3(kSelThreads), 0, s, D, N, k, idx, d);
        return hipGetLastError();
    }
    if (const int per = tau_per(N, k)) {
        const int m = tau_m_per(N, k, per);
        uint32_t *tau = static_cast<uint32_t *>(ws);
        uint32_t *tmin = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) +
                                                      align_up((size_t)M * 4, kAlign));
        const int cfull = N / (kTauThreads * per);
        hipError_t e = launch_fill_u32(reinterpret_cast<int32_t *>(tau), M, 0, s);
        if (e == hipSuccess) {
            if (per == 16)
                hipLaunchKernelGGL(topk_tau_kernel<16>, dim3(cfull, M), dim3(kTauThreads), 0, s, D, N,
                                   m, tau, tmin);
            else
                hipLaunchKernelGGL(topk_tau_kernel<4>, dim3(cfull, M), dim3(kTauThreads), 0, s, D, N,
                                   m, tau, tmin);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            if (per == 16)
                hipLaunchKernelGGL(topk_list_kernel<16>, dim3(M), dim3(kSelThreads), 0, s, D, N, k, tau,
                                   tmin, idx, d);
            else
                hipLaunchKernelGGL(topk_list_kernel<4>, dim3(M), dim3(kSelThreads), 0, s, D, N, k, tau,
                                   tmin, idx, d);
            e = hipGetLastError();
        }
        return e;
    }
    const int nch = (N + kChunk - 1) / kChunk;
    uint32_t *ck = static_cast<uint32_t *>(ws);
    int32_t *ci = reinterpret_cast<int32_t *>(ck + (size_t)M * nch * k);
    hipLaunchKernelGGL(topk_chunk_kernel, dim3(nch, M), dim3(kChunkThreads), 0, s, D, N, k, ck, ci);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(topk_merge_kernel, dim3(M), dim3(kSelThreads), 0, s, nch * k, k, ck, ci, idx,
                       d);
    return hipGetLastError();
}

// Per candidate: score 8, entry 4, overlaps 2 x 4, bound order 4, sorted and unsorted bounds
// 2 x 8, entry in bound order 4 bytes; per query a count 4 and its block counts 2 x 4 bytes
// per block.
size_t rerank_ws_bytes(int nq)
{
    return (size_t)nq * kRerankMaxCand * 44 + 512 + (size_t)nq * (4 + 2 * kBoundMaxBlocks * 4);
}

hipError_t launch_rerank_score(const db_t *db, int nq, const uint32_t *qpack, const uint32_t *acnt,
                               const int32_t *box, const int32_t *tbox, const int32_t *cand,
                               int nc, int k, void *ws, hipStream_t s)
{
    const Geometry &g = db->g;
    const size_t m = (size_t)nq * nc;
    uint64_t *ws_s = static_cast<uint64_t *>(ws);
    int32_t *ws_i = reinterpret_cast<int32_t *>(ws_s + m);
    uint32_t *ws_I = reinterpret_cast<uint32_t *>(ws_i + m);
    int32_t *order = reinterpret_cast<int32_t *>(ws_I + 2 * m);
    double *ubs = reinterpret_cast<double *>(order + m);   // 24 m bytes in: 8-byte aligned
    double *ub = ubs + m;
    int32_t *ents = reinterpret_cast<int32_t *>(ub + m);
    char *tail = static_cast<char *>(ws) + (44 * m + 255) / 256 * 256;
    int32_t *qcount = reinterpret_cast<int32_t *>(tail);
    uint32_t *qbc = reinterpret_cast<uint32_t *>(tail + ((size_t)nq * 4 + 255) / 256 * 256);
    // split: kRC candidates per block with the waves splitting the rows (the bound-ordered
    // rounds, few candidates per query), else 4 kRC per block.
    auto score = [&](int first, int count, const int32_t *ord, const int32_t *en,
                     const int32_t *qc, bool split) {
        const int per = split ? kRC : kRerankPerBlock;
        const int nbq = (count + per - 1) / per;
        const int64_t blocks = (int64_t)nbq * 8 * ((nq + 7) / 8);
#define TDB_RERANK_SCORE(SPLIT_, ALLZR_)                                                            \
    hipLaunchKernelGGL((rerank_score_kernel<SPLIT_, ALLZR_>), dim3((unsigned)blocks), dim3(256), 0, \
                       s, db->planes, db->popcnt, db->box, db->tbox, db->zrange, g.nz, g.Wp,      \
                       g.nxw, g.ny, qpack, acnt, box, tbox, cand, nc, ws_s, ws_i, ws_I, nq, nbq,  \
                       ord, en, qc, first, count)
        const bool allzr = g.nz <= kZStage;
        if (split && allzr) TDB_RERANK_SCORE(4, true);
        else if (split) TDB_RERANK_SCORE(4, false);
        else if (allzr) TDB_RERANK_SCORE(1, true);
        else TDB_RERANK_SCORE(1, false);
#undef TDB_RERANK_SCORE
    };
    int nbx = 0, nby = 0;
    const int nbp = bound_blocks(g, &nbx, &nby);
    const int n1 = (std::max(k, 16) + 15) / 16 * 16;    // scored before the gate
    if (!db->rerank_bound || !db->bcnt || nbp == 0 || k <= 0 || n1 > 64 || nc <= n1) {
        score(0, nc, nullptr, nullptr, nullptr, false);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(query_block_kernel, dim3((unsigned)nq), dim3(256), 0, s, qpack, g.Wp, g.nxw,
                       g.ny, box, nbx, nby, nbp, qbc);
    hipLaunchKernelGGL(rerank_ub_kernel, dim3((unsigned)((int64_t)nq * ((nc + 15) / 16))), dim3(256),
                       0, s, db->bcnt, nbx, nby, nbp, db->popcnt, qbc, box, acnt, cand, nc, nq, ub);
    hipLaunchKernelGGL(rerank_order_kernel, dim3((unsigned)nq), dim3(256), 0, s, ub, cand, nc, order,
                       ubs, ents, ws_s, ws_i);
    score(0, n1, order, ents, nullptr, true);
    hipLaunchKernelGGL(rerank_gate_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, ws_s,
                       order, ubs, nc, n1, k, nq, qcount);
    score(n1, nc - n1, order, ents, qcount, true);
    return hipGetLastError();
}

hipError_t launch_block_counts(const db_t *db, const uint32_t *planes, int64_t n,
                               const int32_t *box, uint16_t *bcnt, hipStream_t s)
{
    int nbx = 0, nby = 0;
    const int nbp = bound_blocks(db->g, &nbx, &nby);
    if (!bcnt || nbp == 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_count_kernel, dim3((unsigned)n), dim3(256), 0, s, planes, db->g.Wp,
                       db->g.nxw, db->g.ny, box, nbx, nby, nbp, bcnt);
    return hipGetLastError();
}

hipError_t launch_rerank_rank(const db_t *db, int nq, const uint32_t *acnt, int nc, int k,
                              int32_t *idx, double *score, db_counts_t *counts, const void *ws,
                              hipStream_t s)
{
    const uint64_t *ws_s = static_cast<const uint64_t *>(ws);
    const int32_t *ws_i = reinterpret_cast<const int32_t *>(ws_s + (size_t)nq * nc);
    const uint32_t *ws_I = reinterpret_cast<const uint32_t *>(ws_i + (size_t)nq * nc);
    hipLaunchKernelGGL(rerank_rank_kernel, dim3(nq), dim3(256), 0, s, db->popcnt, acnt, nc, k, ws_s,
                       ws_i, ws_I, idx, score, counts);
    return hipGetLastError();
}

}  // namespace tdb
