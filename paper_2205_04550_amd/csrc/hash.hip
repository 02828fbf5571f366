// hash.hip — binary codes of latents and Hamming distances (the paper's
// unsupervised hashing query, Sec. 2.3).
//
// The paper's hashing variant is the autoencoder with a "Bi-half" layer
// between encoder and decoder: per latent coordinate, the larger half of a
// batch becomes +1 and the rest -1, so every bit splits the data in two equal
// parts; the query then ranks database codes by L2. For codes in {-1, +1}^D,
// |b_q - b_x|^2 = 4 * Hamming(b_q, b_x), so the ranking is the Hamming one.
// Here a code is stored as D bits (1 = +1), LSB first in uint32 words; the
// database codes use, per coordinate, the lower median of the database as the
// threshold (the Bi-half rule with the whole database as the batch), and a
// query is coded with the same thresholds.
#include "common.hpp"
#include "internal.hpp"

namespace tdb {

// grid dim, 1024 threads: thr[d] = the value of 0-based rank k in ascending
// order of column d of X [n][dim], by four 8-bit radix passes over the
// order-preserving keys of the values (exact: the result is one of the inputs).
__global__ void __launch_bounds__(1024) col_kth_kernel(const float *__restrict__ X, int64_t n,
                                                       int dim, int64_t k, float *__restrict__ thr)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_mask, s_sel[2];
    __shared__ int64_t s_rank;
    const int d = blockIdx.x;
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_mask = 0;
        s_rank = k;
    }
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        const uint32_t prefix = s_prefix, mask = s_mask;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t key = fkey(X[i * dim + d]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        select_bin(hist, (uint32_t)(s_rank + 1), s_sel);   // 1-based rank in this digit
        if (threadIdx.x == 0) {
            s_rank = (int64_t)s_sel[1] - 1;
            s_prefix = prefix | (s_sel[0] << shift);
            s_mask = mask | (255u << shift);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) thr[d] = fkey_inv(s_prefix);
}

hipError_t launch_col_kth(const float *X, int64_t n, int dim, int64_t k, float *thr, hipStream_t s)
{
    hipLaunchKernelGGL(col_kth_kernel, dim3(dim), dim3(1024), 0, s, X, n, dim, k, thr);
    return hipGetLastError();
}

// One thread per code word: bit b of word w of row i is X[i][32w + b] > thr[32w + b].
__global__ void __launch_bounds__(256) binarize_kernel(const float *__restrict__ X, int64_t n,
                                                       int dim, const float *__restrict__ thr,
                                                       uint32_t *__restrict__ codes)
{
    const int words = dim / 32;
    const int64_t total = n * words;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / words;
        const int w = (int)(t - i * words);
        const f32x4 *x = reinterpret_cast<const f32x4 *>(X + i * dim + 32 * w);
        const f32x4 *th = reinterpret_cast<const f32x4 *>(thr + 32 * w);
        uint32_t c = 0;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const f32x4 v = x[g], tv = th[g];
#pragma unroll
            for (int e = 0; e < 4; ++e) c |= (uint32_t)(v[e] > tv[e]) << (4 * g + e);
        }
        codes[t] = c;
    }
}

hipError_t launch_binarize(const float *X, int64_t n, int dim, const float *thr, uint32_t *codes,
                           hipStream_t s)
{
    const int64_t total = n * (dim / 32);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(binarize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, dim, thr,
                       codes);
    return hipGetLastError();
}

constexpr int kHamQ = 32;     // queries per block (codes staged in LDS)
constexpr int kHamMaxW = 32;  // words per code: up to 1024 bits

// grid (ceil(N / 256), ceil(M / kHamQ)): thread = one database code held in
// registers, compared with the block's queries; D[m][n] = popcount(q_m ^ x_n)
// as float (exact: an integer <= 1024).
__global__ void __launch_bounds__(256) hamming_kernel(int M, int N, int words,
                                                      const uint32_t *__restrict__ Q,
                                                      const uint32_t *__restrict__ X,
                                                      float *__restrict__ D)
{
    __shared__ uint32_t sq[kHamQ * kHamMaxW];
    const int q0 = blockIdx.y * kHamQ;
    const int nq = min(kHamQ, M - q0);
    for (int t = threadIdx.x; t < nq * words; t += blockDim.x) sq[t] = Q[(int64_t)q0 * words + t];
    __syncthreads();
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    uint32_t x[kHamMaxW];
#pragma unroll
    for (int w = 0; w < kHamMaxW; ++w) x[w] = w < words ? X[(int64_t)n * words + w] : 0u;
    for (int j = 0; j < nq; ++j) {
        uint32_t h = 0;
#pragma unroll
        for (int w = 0; w < kHamMaxW; ++w)
            if (w < words) h += popc(sq[j * words + w] ^ x[w]);
        D[(int64_t)(q0 + j) * N + n] = (float)h;
    }
}

hipError_t launch_hamming(int M, int N, int words, const uint32_t *Q, const uint32_t *X, float *D,
                          hipStream_t s)
{
    hipLaunchKernelGGL(hamming_kernel, dim3((unsigned)((N + 255) / 256), (unsigned)((M + kHamQ - 1) / kHamQ)),
                       dim3(256), 0, s, M, N, words, Q, X, D);
    return hipGetLastError();
}

// ---- the Bi-half layer of a training step ----

// One thread per coordinate d of a batch U [B][D]: rank of row i is the number
// of rows ranking before it by (value desc, row asc); the first floor(B / 2)
// ranks give +1, the others -1.
template <typename T>
__global__ void __launch_bounds__(256) bihalf_fwd_kernel(int B, int D, const T *__restrict__ U,
                                                         T *__restrict__ out)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    const int half = B / 2;
    for (int i = 0; i < B; ++i) {
        const T u = U[(int64_t)i * D + d];
        int rank = 0;
        for (int j = 0; j < B; ++j) {
            const T v = U[(int64_t)j * D + d];
            rank += (v > u) || (v == u && j < i);
        }
        out[(int64_t)i * D + d] = rank < half ? (T)1 : (T)-1;
    }
}

// dU = G + gamma * ((U - Bc) / (B * D)), evaluated in that order in T: the
// straight-through gradient plus the pull of each value towards its code.
template <typename T>
__global__ void __launch_bounds__(256) bihalf_bwd_kernel(int64_t total, T den, T gamma,
                                                         const T *__restrict__ U,
                                                         const T *__restrict__ Bc,
                                                         const T *__restrict__ G,
                                                         T *__restrict__ dU)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const T diff = U[t] - Bc[t];
        const T scaled = diff / den;
        const T pull = gamma * scaled;
        dU[t] = G[t] + pull;
    }
}

hipError_t launch_bihalf_fwd(bool f64, int B, int D, const void *U, void *out, hipStream_t s)
{
    const dim3 grid((unsigned)((D + 255) / 256));
    if (f64)
        hipLaunchKernelGGL(bihalf_fwd_kernel<double>, grid, dim3(256), 0, s, B, D,
                           static_cast<const double *>(U), static_cast<double *>(out));
    else
        hipLaunchKernelGGL(bihalf_fwd_kernel<float>, grid, dim3(256), 0, s, B, D,
                           static_cast<const float *>(U), static_cast<float *>(out));
    return hipGetLastError();
}

hipError_t launch_bihalf_bwd(bool f64, int B, int D, double gamma, const void *U, const void *Bc,
                             const void *G, void *dU, hipStream_t s)
{
    const int64_t total = (int64_t)B * D;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const double den = (double)B * (double)D;
    if (f64)
        hipLaunchKernelGGL(bihalf_bwd_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, total,
                           den, gamma, static_cast<const double *>(U),
                           static_cast<const double *>(Bc), static_cast<const double *>(G),
                           static_cast<double *>(dU));
    else
        hipLaunchKernelGGL(bihalf_bwd_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, total,
                           (float)den, (float)gamma, static_cast<const float *>(U),
                           static_cast<const float *>(Bc), static_cast<const float *>(G),
                           static_cast<float *>(dU));
    return hipGetLastError();
}

}  // namespace tdb
