// nn.hip — encoder / decoder kernels for the embedding search (C ABI in include/tumornn.h).
//
// The paper's autoencoder (Sec. 2.4 "Implementation"): strided 3-D
// convolutions (stride 2, kernel 3), a linear layer to the latent, and a
// mirrored decoder of strided transposed convolutions; trained to reconstruct
// its input. The forward pass runs on the matrix cores as implicit GEMMs: the
// first layer (mean-pooled labels or packed masks in, whose pooled values k/8
// are exact in BF16) on BF16 16x16x32 products, the later convolutions with
// Ci % 4 == 0 and the linear layers on FP32 16x16x4 / 32x32x2 products (each
// product exact in FP32, only the summation order differs from a direct sum).
// The backward kernels and the FP64 instantiation used by finite-difference
// checks are direct convolutions on the vector ALUs: one thread per output (or
// input, for the adjoint) voxel with block-uniform channel and batch indices.
// Weight gradients reduce in two deterministic stages. Kernels are templates
// over the activation type T (float, or double) and the weight storage type
// (bfloat16 bits, float or double); accumulation is in T.
#include <hip/hip_runtime.h>

#include "../../include/tumornn.h"
#include "common.hpp"
#include "internal.hpp"

namespace tdb {

__device__ __forceinline__ float ld_w(const uint16_t *p, int64_t i)
{
    return __uint_as_float((uint32_t)p[i] << 16);
}
__device__ __forceinline__ float ld_w(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ double ld_w(const double *p, int64_t i) { return p[i]; }

template <class T>
__device__ __forceinline__ T wsum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// ---- convolution, kernel 3, stride 2, padding 1 ------------------------------------------

constexpr int kCB = 8;   // output channels per thread: each input tap is loaded once for all
constexpr int kCC = 8;   // channels of the other side staged in LDS per step

// Weights of kCB output channels x kCC input channels, laid out [cc][tap][c] so that
// one tap's kCB weights are contiguous (vector reads, same address across the wave).
// `other` = the summed-over channel index base, `own` = this block's channel base.
template <class T, class WT, int CB = kCB>
__device__ __forceinline__ void stage_weights(T *wsh, const WT *__restrict__ Wt, int Ci, int Co,
                                              int own0, int nown, int other0, int nother,
                                              bool own_is_co)
{
    for (int t = threadIdx.x; t < kCC * 27 * CB; t += blockDim.x) {
        const int c = t % CB, tap = (t / CB) % 27, cc = t / (CB * 27);
        T v = T(0);
        if (c < nown && cc < nother) {
            const int own = own0 + c, oth = other0 + cc;
            const int co = own_is_co ? own : oth;
            const int ci = own_is_co ? oth : own;
            v = (T)ld_w(Wt, ((int64_t)co * Ci + ci) * 27 + tap);
        }
        wsh[t] = v;
    }
}

// grid (ceil(B*OD*OH*OW / (256 VX)), ceil(Co / CB)): one thread per (sample, VX
// adjacent output voxels along x) and CB output channels, so small late layers
// still fill whole waves. Each weight read from LDS feeds VX * CB multiply-adds
// and neighbouring outputs share their common input taps.
template <class T, class WT, int CB, int VX>
__global__ void __launch_bounds__(256) conv_fwd_kernel(int B, int Ci, int Co, int D, int H, int W,
                                                       const T *__restrict__ X,
                                                       const WT *__restrict__ Wt,
                                                       const T *__restrict__ bias, int relu,
                                                       T *__restrict__ Y)
{
    __shared__ T wsh[kCC * 27 * CB];
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int osp = OD * OH * OW;
    const int gpr = OW / VX;                          // thread groups per output row
    const int gsp = OD * OH * gpr;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = t < (int64_t)B * gsp;
    const int64_t tt = active ? t : 0;
    const int b = (int)(tt / gsp);
    const int gi = (int)(tt - (int64_t)b * gsp);
    const int ow0 = (gi % gpr) * VX, oh = (gi / gpr) % OH, od = gi / (gpr * OH);
    const int co0 = blockIdx.y * CB;
    const int nco = min(CB, Co - co0);
    const int64_t isp = (int64_t)D * H * W;
    T acc[VX][CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const T b0 = bias ? bias[min(co0 + c, Co - 1)] : T(0);
#pragma unroll
        for (int v = 0; v < VX; ++v) acc[v][c] = b0;
    }
    for (int ci0 = 0; ci0 < Ci; ci0 += kCC) {
        const int ncc = min(kCC, Ci - ci0);
        __syncthreads();
        stage_weights<T, WT, CB>(wsh, Wt, Ci, Co, co0, nco, ci0, ncc, true);
        __syncthreads();
        for (int cc = 0; cc < ncc; ++cc) {
            const T *x = X + ((int64_t)b * Ci + ci0 + cc) * isp;
            const T *w = wsh + cc * 27 * CB;
            // Not unrolled over kd: keeps the live weights to one 3x3 plane.
#pragma unroll 1
            for (int kd = 0; kd < 3; ++kd) {
                const int id = 2 * od + kd - 1;
#pragma unroll
                for (int kh = 0; kh < 3; ++kh) {
                    const int ih = 2 * oh + kh - 1;
                    const bool row_in = id >= 0 && id < D && ih >= 0 && ih < H;
                    const int64_t row = row_in ? ((int64_t)id * H + ih) * W : 0;
                    T xr[2 * VX + 1];
#pragma unroll
                    for (int j = 0; j < 2 * VX + 1; ++j) {
                        const int iw = 2 * ow0 - 1 + j;
                        const bool in = row_in && iw >= 0 && iw < W;
                        xr[j] = in ? x[row + iw] : T(0);
                    }
#pragma unroll
                    for (int kw = 0; kw < 3; ++kw) {
                        const T *wt = w + (kd * 9 + kh * 3 + kw) * CB;
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            const T wv = wt[c];
#pragma unroll
                            for (int v = 0; v < VX; ++v) acc[v][c] += wv * xr[2 * v + kw];
                        }
                    }
                }
            }
        }
    }
    if (!active) return;
    const int o0 = (od * OH + oh) * OW + ow0;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        if (c >= nco) break;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            T r = acc[v][c];
            if (relu && r < T(0)) r = T(0);
            Y[((int64_t)b * Co + co0 + c) * osp + o0 + v] = r;
        }
    }
}

// Forward on the FP32 matrix cores for float activations (Ci % 4 == 0, W % 4 ==
// 0): an implicit GEMM Y[co][voxel] = sum over (tap, ci) of W[co][ci][tap]
// X[ci][voxel + tap], each product exact in FP32 as with FMA (only the summation
// order differs). A tile is a TD x TH x TW box of output voxels of one sample
// with all output channels; a block takes npb tiles in turn. Per tile and chunk
// of four input channels (a stage) it stages in LDS the input patch, (2TD+1) x
// (2TH+1) rows of 2TW+8 floats (the 2TW+1 needed, widened to whole aligned
// 16-byte groups; zeros outside the volume), and the chunk's weights (bf16
// widened to float); the next stage's loads are in flight in registers while
// the current one is multiplied. Each wave owns MT tiles of 16 voxels along x
// and NT tiles of 16 output channels; one 16 x 16 x 4 product takes the four
// channels of one tap, lane l giving channel l / 16 for voxel (or output
// channel) l % 16.
__device__ __forceinline__ void ld_w2(const uint16_t *p, float *o)
{
    const uint32_t u = *reinterpret_cast<const uint32_t *>(p);
    o[0] = __uint_as_float(u << 16);
    o[1] = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void ld_w2(const float *p, float *o)
{
    const float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x;
    o[1] = v.y;
}

template <int TD, int TH, int TW, int NT>
struct ConvTile {
    static constexpr int PWA = 2 * TW + 8, SEGS = PWA / 4, PH = 2 * TH + 1, PD = 2 * TD + 1;
    static constexpr int PROWS = PD * PH, PVA = PROWS * PWA;
    static constexpr int NX4 = 4 * PROWS * SEGS;              // float4 groups of a stage
    static constexpr int NW = NT * 16 * 108;                  // weights of a stage
    static constexpr int XB = (NX4 + 255) / 256, WB = (NW / 2 + 255) / 256;   // WB: pairs
    static constexpr int WALL = 4096;                         // floats: all weights at once
    static constexpr int WLDS = NW > WALL ? NW : WALL;
    static constexpr int LDS = 4 * PVA + WLDS;                // floats
};

// WALL: every weight of the layer sits in LDS for the whole block ([co][ci][tap], rows of
// 27 Ci + 1 floats), staged once; otherwise each stage brings its chunk's weights
// ([co][4][27], rows of 108).
template <class WT, int TD, int TH, int TW, int MT, int NT, bool WALL>
__global__ void __launch_bounds__(256) conv_mfma_kernel(int Ci, int Co, int D, int H, int W,
                                                        int tiles_h, int tiles_w, int T, int npb,
                                                        const float *__restrict__ X,
                                                        const WT *__restrict__ Wt,
                                                        const float *__restrict__ bias, int relu,
                                                        float *__restrict__ Y)
{
    static_assert(TD * TH * TW == 64 * MT, "a wave owns MT tiles of 16 voxels");
    using G = ConvTile<TD, TH, TW, NT>;
    constexpr int PWA = G::PWA, SEGS = G::SEGS, PH = G::PH, PROWS = G::PROWS, PVA = G::PVA;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS];
    float *xs = lds;
    float *ws = lds + 4 * PVA;
    const int wrow = WALL ? 27 * Ci + 1 : 108;
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kq = lane >> 4;
    const int b = blockIdx.y;
    int t0 = blockIdx.x * npb;
    if (T % (8 * npb) == 0) t0 = (blockIdx.x % 8) * (T / 8) + (blockIdx.x / 8) * npb;
    const int nt_blk = min(npb, T - t0);
    const int nc = Ci / 4, K = nt_blk * nc;
    int vb[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int v = (wave * MT + m) * 16 + (lane & 15);
        const int z = v / (TH * TW), y = (v / TW) % TH, x = v % TW;
        vb[m] = kq * PVA + (2 * z * PH + 2 * y) * PWA + 2 * x + 3;
    }
    const int HW = H * W;
    const int isp = D * HW;
    const float *Xb = X + (int64_t)b * Ci * isp;
    // Per staged float4 of this thread: patch row (z, y), 16-byte group seg and channel,
    // packed, and its offset from the patch origin (the same for every stage).
    int pk[G::XB], rel[G::XB];
#pragma unroll
    for (int j = 0; j < G::XB; ++j) {
        const int e = j * 256 + tid;
        const int row = e / SEGS, seg = e - row * SEGS;
        const int ci = row / PROWS, rr = row - ci * PROWS;
        const int z = rr / PH, y = rr % PH;
        pk[j] = e < G::NX4 ? z | (y << 8) | (seg << 16) : -1;
        rel[j] = ci * isp + z * HW + y * W + 4 * seg;
    }
    if (WALL) {                                 // all weights, once
        for (int e = tid; e < NT * 16 * 27 * Ci; e += 256) {
            const int co = e / (27 * Ci), r = e - co * (27 * Ci);
            ws[co * wrow + r] = co < Co ? ld_w(Wt, (int64_t)co * 27 * Ci + r) : 0.f;
        }
    }
    f32x4 xin[G::XB];
    float wv[WALL ? 1 : G::WB][2];
    // Loads of stage k: tile t0 + k / nc, input channels 4 (k % nc) .. + 3. Patch origin:
    // row (z, y) = input (2 od0 - 1 + z, 2 oh0 - 1 + y); column c = input x 2 ow0 - 4 + c,
    // so tap kw of output x-offset ox sits at column 2 ox + kw + 3.
    auto fetch = [&](int k) {
        const int t = t0 + k / nc, c0 = 4 * (k % nc);
        const int tw = t % tiles_w, th = (t / tiles_w) % tiles_h, td = t / (tiles_w * tiles_h);
        const int iz0 = 2 * td * TD - 1, iy0 = 2 * th * TH - 1, ix0 = 2 * tw * TW - 4;
        const float *org = Xb + (int64_t)c0 * isp + (int64_t)iz0 * HW + iy0 * W + ix0;
        // Branch-free: an element outside the volume loads the sample's first group
        // (always valid) and is replaced by zeros.
#pragma unroll
        for (int j = 0; j < G::XB; ++j) {
            const int z = pk[j] & 0xff, y = (pk[j] >> 8) & 0xff, seg = (pk[j] >> 16) & 0xff;
            const bool ok = pk[j] >= 0 && (unsigned)(iz0 + z) < (unsigned)D &&
                            (unsigned)(iy0 + y) < (unsigned)H && (unsigned)(ix0 + 4 * seg) < (unsigned)W;
            const f32x4 t = *reinterpret_cast<const f32x4 *>(ok ? org + rel[j] : Xb);
            xin[j] = ok ? t : (f32x4){0.f, 0.f, 0.f, 0.f};
        }
        if (!WALL) {
            // Weights in pairs (r even; 108 per output channel and chunk, so a pair never
            // straddles two channels, and Ci % 4 == 0 keeps the pair 2-element aligned).
#pragma unroll
            for (int j = 0; j < G::WB; ++j) {
                const int e = 2 * (j * 256 + tid);
                const int co = e / 108, r = e - co * 108;
                wv[j][0] = wv[j][1] = 0.f;
                if (e < G::NW && co < Co) ld_w2(Wt + ((int64_t)co * Ci + c0) * 27 + r, wv[j]);
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int j = 0; j < G::XB; ++j) {
            const int e = j * 256 + tid;
            if (e < G::NX4) *reinterpret_cast<f32x4 *>(&xs[4 * e]) = xin[j];
        }
        if (!WALL) {
#pragma unroll
            for (int j = 0; j < G::WB; ++j) {
                const int e = 2 * (j * 256 + tid);
                if (e < G::NW) {
                    ws[e] = wv[j][0];
                    ws[e + 1] = wv[j][1];
                }
            }
        }
    };
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int64_t osp = (int64_t)OD * OH * OW;
    if (K > 0) fetch(0);
    for (int k = 0; k < K; ++k) {
        stash();
        __syncthreads();
        if (k + 1 < K) fetch(k + 1);
        const float *wq = ws + (lane & 15) * wrow + (WALL ? 4 * (k % nc) + kq : kq) * 27;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int toff = ((tap / 9) * PH + (tap / 3) % 3) * PWA + tap % 3;
            float a[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) a[n] = wq[n * 16 * wrow + tap];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const float bv = xs[vb[m] + toff];
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[n], bv, acc[m][n], 0, 0, 0);
            }
        }
        if (k % nc == nc - 1) {                 // last chunk of this tile: write it out
            const int t = t0 + k / nc;
            const int tw = t % tiles_w, th = (t / tiles_w) % tiles_h, td = t / (tiles_w * tiles_h);
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int v = (wave * MT + m) * 16 + (lane & 15);
                const int oz = td * TD + v / (TH * TW), oy = th * TH + (v / TW) % TH;
                const int ox = tw * TW + v % TW;
                const bool ok = oz < OD && oy < OH && ox < OW;
                const int64_t o = ((int64_t)oz * OH + oy) * OW + ox;
#pragma unroll
                for (int n = 0; n < NT; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int co = n * 16 + 4 * kq + r;
                        if (ok && co < Co) {
                            float y = acc[m][n][r] + (bias ? bias[co] : 0.f);
                            if (relu && y < 0.f) y = 0.f;
                            Y[((int64_t)b * Co + co) * osp + o] = y;
                        }
                        acc[m][n][r] = 0.f;
                    }
            }
        }
        __syncthreads();                        // the next stash overwrites the stage
    }
}

// Adjoint map: grid (ceil(B*D*H*W / 256), ceil(Ci / kCB)); one thread per (sample,
// input voxel) and kCB input channels (each dY tap is loaded once for all of them).
// Threads are numbered by parity class: the voxels of one sample with the same
// (z, y, x) parities are consecutive, so the lanes of a wave share the set of taps
// that reach them (1 or 2 per axis) and skip the others together.
template <class T, class WT>
__global__ void __launch_bounds__(256) conv_bwd_data_kernel(int B, int Ci, int Co, int D, int H,
                                                            int W, const T *__restrict__ dY,
                                                            const WT *__restrict__ Wt,
                                                            const T *__restrict__ bias, int relu,
                                                            T *__restrict__ dX)
{
    __shared__ T wsh[kCC * 27 * kCB];
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int osp = OD * OH * OW;
    const int isp = D * H * W;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = t < (int64_t)B * isp;
    const int64_t tt = active ? t : 0;
    const int b = (int)(tt / isp);
    const int r = (int)(tt - (int64_t)b * isp);
    const int cls = r / osp, jv = r - cls * osp;
    const int iw = 2 * (jv % OW) + (cls & 1);
    const int ih = 2 * ((jv / OW) % OH) + ((cls >> 1) & 1);
    const int id = 2 * (jv / (OW * OH)) + (cls >> 2);
    const int i = (id * H + ih) * W + iw;
    const int ci0 = blockIdx.y * kCB;
    const int nci = min(kCB, Ci - ci0);
    T acc[kCB];
#pragma unroll
    for (int c = 0; c < kCB; ++c) acc[c] = bias ? bias[min(ci0 + c, Ci - 1)] : T(0);
    for (int co0 = 0; co0 < Co; co0 += kCC) {
        const int ncc = min(kCC, Co - co0);
        __syncthreads();
        stage_weights(wsh, Wt, Ci, Co, ci0, nci, co0, ncc, false);
        __syncthreads();
        for (int cc = 0; cc < ncc; ++cc) {
            const T *dy = dY + ((int64_t)b * Co + co0 + cc) * osp;
            const T *w = wsh + cc * 27 * kCB;
#pragma unroll
            for (int kd = 0; kd < 3; ++kd) {
                const int td = id + 1 - kd;
                if (td < 0 || (td & 1) || (td >> 1) >= OD) continue;
#pragma unroll
                for (int kh = 0; kh < 3; ++kh) {
                    const int th = ih + 1 - kh;
                    if (th < 0 || (th & 1) || (th >> 1) >= OH) continue;
#pragma unroll
                    for (int kw = 0; kw < 3; ++kw) {
                        const int tw = iw + 1 - kw;
                        if (tw < 0 || (tw & 1) || (tw >> 1) >= OW) continue;
                        const T g = dy[((td >> 1) * OH + (th >> 1)) * OW + (tw >> 1)];
                        const T *wt = w + (kd * 9 + kh * 3 + kw) * kCB;
#pragma unroll
                        for (int c = 0; c < kCB; ++c) acc[c] += wt[c] * g;
                    }
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
        if (c >= nci) break;
        T v = acc[c];
        if (relu && v < T(0)) v = T(0);
        dX[((int64_t)b * Ci + ci0 + c) * isp + i] = v;
    }
}

constexpr int kWgChunk = 4096;  // (batch, output voxel) positions per weight-gradient block

// Stage 1: grid (chunks, Ci, ceil(Co / CB)). partial [chunks][Co][Ci][28]: 27 taps + sum
// of dY. A thread takes CB output channels at once, so each input tap it loads feeds CB
// products; each (co, ci, tap) sum is formed in the same order whatever CB is.
template <class T, int CB>
__global__ void __launch_bounds__(256) conv_bwd_weight_partial(int B, int Ci, int Co, int D, int H,
                                                               int W, const T *__restrict__ X,
                                                               const T *__restrict__ dY,
                                                               T *__restrict__ partial)
{
    __shared__ T red[4][CB][28];
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int osp = OD * OH * OW;
    const int64_t isp = (int64_t)D * H * W;
    const int co0 = blockIdx.z * CB, ci = blockIdx.y;
    const int64_t P = (int64_t)B * osp;
    const int64_t p0 = (int64_t)blockIdx.x * kWgChunk;
    const int64_t p1 = p0 + kWgChunk < P ? p0 + kWgChunk : P;
    T acc[CB][28];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int k = 0; k < 28; ++k) acc[c][k] = T(0);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int b = (int)(p / osp);
        const int o = (int)(p - (int64_t)b * osp);
        const int ow = o % OW, oh = (o / OW) % OH, od = o / (OW * OH);
        T g[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c)
            g[c] = co0 + c < Co ? dY[((int64_t)b * Co + co0 + c) * osp + o] : T(0);
        const T *x = X + ((int64_t)b * Ci + ci) * isp;
#pragma unroll
        for (int kd = 0; kd < 3; ++kd) {
            const int id = 2 * od + kd - 1;
#pragma unroll
            for (int kh = 0; kh < 3; ++kh) {
                const int ih = 2 * oh + kh - 1;
#pragma unroll
                for (int kw = 0; kw < 3; ++kw) {
                    const int iw = 2 * ow + kw - 1;
                    const bool in = id >= 0 && id < D && ih >= 0 && ih < H && iw >= 0 && iw < W;
                    // Out-of-range taps read element 0 (always valid) and count as zero.
                    const int64_t off = in ? ((int64_t)id * H + ih) * W + iw : 0;
                    const T xv = in ? x[off] : T(0);
#pragma unroll
                    for (int c = 0; c < CB; ++c) acc[c][kd * 9 + kh * 3 + kw] += g[c] * xv;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c][27] += g[c];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int k = 0; k < 28; ++k) {
            const T sm = wsum(acc[c][k]);
            if (lane == 0) red[wave][c][k] = sm;
        }
    __syncthreads();
    for (int t = threadIdx.x; t < CB * 28; t += blockDim.x) {
        const int c = t / 28, k = t - c * 28;
        if (co0 + c >= Co) continue;
        const T sm = ((red[0][c][k] + red[1][c][k]) + red[2][c][k]) + red[3][c][k];
        partial[(((int64_t)blockIdx.x * Co + co0 + c) * Ci + ci) * 28 + k] = sm;
    }
}

// Stage 2: one thread per (co, ci, tap) sums the chunks in order.
template <class T>
__global__ void conv_bwd_weight_final(int nchunks, int Ci, int Co, const T *__restrict__ partial,
                                      T *__restrict__ dW, T *__restrict__ dbias)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Co * Ci * 28) return;
    const int k = t % 28;
    const int cc = t / 28;  // co * Ci + ci
    T s = T(0);
    for (int c = 0; c < nchunks; ++c)
        s += partial[((int64_t)c * Co * Ci + cc) * 28 + k];
    if (k < 27)
        dW[(int64_t)cc * 27 + k] = s;
    else if (dbias && (cc % Ci) == 0)
        dbias[cc / Ci] = s;
}

// ---- linear ---------------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(256) linear_bwd_weight_kernel(int B, int In, int Out,
                                                                const T *__restrict__ X,
                                                                const T *__restrict__ dY,
                                                                T *__restrict__ dW,
                                                                T *__restrict__ dbias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= In) return;
    T acc = T(0);
    for (int b = 0; b < B; ++b) acc += dY[(int64_t)b * Out + j] * X[(int64_t)b * In + i];
    dW[(int64_t)j * In + i] = acc;
    if (dbias && i == 0) {
        T s = T(0);
        for (int b = 0; b < B; ++b) s += dY[(int64_t)b * Out + j];
        dbias[j] = s;
    }
}

// out[c] = sum over (b, s) of X[b][c][s], in two fixed-order stages:
// grid (chunks, C) partial sums over kCsChunk consecutive (b, s) positions, then
// one thread per channel adds the chunks in order.
constexpr int kCsChunk = 16384;

template <class T>
__global__ void __launch_bounds__(256) channel_sum_partial(int B, int C, int64_t S,
                                                           const T *__restrict__ X,
                                                           T *__restrict__ partial)
{
    __shared__ T red[4];
    const int c = blockIdx.y;
    const int64_t P = (int64_t)B * S;
    const int64_t p0 = (int64_t)blockIdx.x * kCsChunk;
    const int64_t p1 = p0 + kCsChunk < P ? p0 + kCsChunk : P;
    T acc = T(0);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int64_t b = p / S, sidx = p - b * S;
        acc += X[(b * C + c) * S + sidx];
    }
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(int64_t)c * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <class T>
__global__ void channel_sum_final(int C, int nchunks, const T *__restrict__ partial,
                                  T *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    T s = T(0);
    for (int i = 0; i < nchunks; ++i) s += partial[(int64_t)c * nchunks + i];
    out[c] = s;
}

// ---- tiled GEMM for the linear layers (vector ALUs) ------------------------------------------
//
// C[m][n] = act(bias[n] + sum_k A[m][k] * B(k, n)), A row-major [M][K]; B is either
// [N][K] (K contiguous: forward, x W^T) or [K][N] (N contiguous: input gradient,
// dY W). 256 threads, tile 32 x 64 x 32 staged in LDS; each thread 2 x 4 outputs.
constexpr int kLM = 32, kLN = 64, kLK = 32;

template <class T, class WT, bool B_KN>
__global__ void __launch_bounds__(256) linear_gemm_kernel(int M, int N, int K,
                                                          const T *__restrict__ A,
                                                          const WT *__restrict__ Bm,
                                                          const T *__restrict__ bias, int relu,
                                                          T *__restrict__ C)
{
    __shared__ T As[kLK][kLM + 1];
    __shared__ T Bs[kLK][kLN + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * kLM, n0 = blockIdx.x * kLN;
    T acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
    for (int k0 = 0; k0 < K; k0 += kLK) {
        for (int t = threadIdx.x; t < kLM * kLK; t += blockDim.x) {
            const int mm = t / kLK, kk = t % kLK;
            const int m = m0 + mm, k = k0 + kk;
            As[kk][mm] = (m < M && k < K) ? A[(int64_t)(m < M ? m : 0) * K + (k < K ? k : 0)] : T(0);
        }
        for (int t = threadIdx.x; t < kLN * kLK; t += blockDim.x) {
            int nn, kk;
            if (B_KN) {          // N contiguous in memory
                nn = t % kLN;
                kk = t / kLN;
            } else {             // K contiguous in memory
                kk = t % kLK;
                nn = t / kLK;
            }
            const int n = n0 + nn, k = k0 + kk;
            const bool in = n < N && k < K;
            const int nc = in ? n : 0, kc = in ? k : 0;
            const T v = (T)ld_w(Bm, B_KN ? (int64_t)kc * N + nc : (int64_t)nc * K + kc);
            Bs[kk][nn] = in ? v : T(0);
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kLK; ++kk) {
            const T a0 = As[kk][ty * 2], a1 = As[kk][ty * 2 + 1];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T bv = Bs[kk][tx + 16 * j];
                acc[0][j] += a0 * bv;
                acc[1][j] += a1 * bv;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = m0 + ty * 2 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx + 16 * j;
            if (n >= N) continue;
            T v = acc[i][j] + (bias ? bias[n] : T(0));
            if (relu && v < T(0)) v = T(0);
            C[(int64_t)m * N + n] = v;
        }
    }
}

// Forward C[m][n] = act(bias[n] + sum_k A[m][k] W[n][k]) in float on the FP32
// matrix cores (products exact in FP32 as with FMA; only the summation order
// differs). Block tile 64 x 64, four waves of 32 x 32; K in steps of 32 staged
// in LDS with the next step's loads in flight. In product s of a step, lane l
// supplies row (or column) l % 32 at k = 16 (l / 32) + s, so a lane reads 16
// consecutive k of its row as four 16-byte LDS loads. Needs K % 4 == 0.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMM = 64, kMK = 64, kMPad = kMK + 4;

__device__ __forceinline__ f32x4 ld4_w(const float *p) { return *reinterpret_cast<const f32x4 *>(p); }
__device__ __forceinline__ f32x4 ld4_w(const uint16_t *p)
{
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    return (f32x4){__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                   __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
}

// SPLIT: block z multiplies only k in [z kc, (z + 1) kc) (kc a multiple of kMK) and writes its
// raw sums to C + z M N (no bias, no ReLU); linear_split_final_kernel adds the slices.
template <class WT, bool B_KN, bool SPLIT = false>
__global__ void __launch_bounds__(512) linear_mfma_kernel(int M, int N, int K,
                                                          const float *__restrict__ A,
                                                          const WT *__restrict__ Wt,
                                                          const float *__restrict__ bias, int relu,
                                                          float *__restrict__ C, int kc = 0)
{
    const int kb = SPLIT ? blockIdx.z * kc : 0, ke = SPLIT ? min(K, kb + kc) : K;
    __shared__ __attribute__((aligned(16))) float As[kMM * kMPad];
    __shared__ __attribute__((aligned(16))) float Bs[kMM * kMPad];
    __shared__ float red[4 * 16 * 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Eight waves: kh = wave / 4 takes half of each 32-wide K step, so twice as many
    // waves share a tile; the two halves are added at the end (fixed order).
    const int kh = wave >> 2, w4 = wave & 3;
    const int wm = w4 >> 1, wn = w4 & 1, h = lane >> 5, r32 = lane & 31;
    const int m0 = blockIdx.y * kMM, n0 = blockIdx.x * kMM;
    // Staging: 64 rows x kMK / 4 float4 per operand, kSt of each per thread. With B_KN
    // the weights are [K][N] (the input gradient dY W): four consecutive n of one k.
    constexpr int kF4 = kMK / 4, kRows = 512 / kF4, kSt = kMM / kRows;
    static_assert(kSt == kMK / 32, "both operands take kSt passes");
    const int srow = tid / kF4, sk = (tid % kF4) * 4;    // + kRows j rows
    const int bk = tid >> 4, bq = (tid & 15) * 4;        // + 32 j k
    f32x4 pa[kSt], pb[kSt];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int j = 0; j < kSt; ++j) {
            const int k = k0 + sk;
            const int m = m0 + srow + kRows * j, n = n0 + srow + kRows * j;
            pa[j] = (m < M && k < ke) ? ld4_w(A + (int64_t)m * K + k) : (f32x4){0.f, 0.f, 0.f, 0.f};
            if (B_KN) {
                const int kr = k0 + bk + 32 * j, nb = n0 + bq;
                pb[j] = (kr < ke && nb < N) ? ld4_w(Wt + (int64_t)kr * N + nb)
                                            : (f32x4){0.f, 0.f, 0.f, 0.f};
            } else {
                pb[j] = (n < N && k < ke) ? ld4_w(Wt + (int64_t)n * K + k)
                                          : (f32x4){0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += kMK) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSt; ++j) {
            *reinterpret_cast<f32x4 *>(&As[(srow + kRows * j) * kMPad + sk]) = pa[j];
            if (B_KN) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[(bq + e) * kMPad + bk + 32 * j] = pb[j][e];
            } else {
                *reinterpret_cast<f32x4 *>(&Bs[(srow + kRows * j) * kMPad + sk]) = pb[j];
            }
        }
        __syncthreads();
        if (k0 + kMK < ke) fetch(k0 + kMK);
        // In product s of this wave's half, lane l supplies row (or column) l % 32 at
        // k = (kMK / 2) (l / 32) + (kMK / 4) kh + s.
        const float *ar = &As[(wm * 32 + r32) * kMPad + (kMK / 2) * h + (kMK / 4) * kh];
        const float *br = &Bs[(wn * 32 + r32) * kMPad + (kMK / 2) * h + (kMK / 4) * kh];
#pragma unroll
        for (int q = 0; q < kMK / 16; ++q) {
            const f32x4 a = *reinterpret_cast<const f32x4 *>(ar + 4 * q);
            const f32x4 b = *reinterpret_cast<const f32x4 *>(br + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], acc, 0, 0, 0);
        }
    }
    if (kh == 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) red[(w4 * 16 + r) * 64 + lane] = acc[r];
    }
    __syncthreads();
    if (kh == 1) return;
    const int n = n0 + wn * 32 + r32;
    if (n >= N) return;
    const float bn = bias ? bias[n] : 0.f;
    if (SPLIT) C += (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (m < M) {
            float v = acc[r] + red[(w4 * 16 + r) * 64 + lane];
            if (!SPLIT) {
                v += bn;
                if (relu && v < 0.f) v = 0.f;
            }
            C[(int64_t)m * N + n] = v;
        }
    }
}

// Y[m][n] = act(sum over z < S of P[z][m][n], in that order, + bias[n]): the slices of a
// split linear_mfma_kernel. With S = 1 the result is the unsplit kernel's bit for bit.
__global__ void linear_split_final_kernel(int64_t MN, int N, int S, const float *__restrict__ P,
                                          const float *__restrict__ bias, int relu,
                                          float *__restrict__ Y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < MN;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = P[i];
        for (int z = 1; z < S; ++z) v += P[z * MN + i];
        v += bias ? bias[i % N] : 0.f;
        Y[i] = relu && v < 0.f ? 0.f : v;
    }
}

// ---- elementwise, loss, optimiser ---------------------------------------------------------

template <class T>
__global__ void relu_bwd_kernel(int64_t n, const T *__restrict__ Y, const T *__restrict__ dY,
                                T *__restrict__ dX)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dX[i] = Y[i] > T(0) ? dY[i] : T(0);
}

constexpr int kMseBlocks = 512;

template <class T>
__global__ void __launch_bounds__(256) mse_partial_kernel(int64_t n, const T *__restrict__ A,
                                                          const T *__restrict__ B,
                                                          T *__restrict__ partial)
{
    __shared__ T red[4];
    T acc = T(0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T d = A[i] - B[i];
        acc += d * d;
    }
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <class T>
__global__ void mse_final_kernel(int nb, int64_t n, const T *__restrict__ partial,
                                 T *__restrict__ loss)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        T s = T(0);
        for (int i = 0; i < nb; ++i) s += partial[i];
        loss[0] = s / (T)n;
    }
}

template <class T>
__global__ void mse_bwd_kernel(int64_t n, const T *__restrict__ A, const T *__restrict__ B,
                               const T *__restrict__ g, T *__restrict__ dA)
{
    const T scale = g[0] * T(2) / (T)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dA[i] = scale * (A[i] - B[i]);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);  // quiet NaN
    const uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

// Two floats -> two bfloat16 values, round to nearest even, lo in bits 0..15 (one
// v_cvt_pk_bf16_f32). FP32 denormals are kept in these kernels (denormal mode 3), so
// every non-NaN input gives f32_to_bf16_rne's bits; a NaN stays a NaN.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_rne(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}

__global__ void adam_kernel(int64_t n, float *__restrict__ w, float *__restrict__ m,
                            float *__restrict__ v, const float *__restrict__ g,
                            uint16_t *__restrict__ wb, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (wb) wb[i] = f32_to_bf16_rne(wi);
    }
}

__global__ void to_bf16_kernel(int64_t n, const float *__restrict__ x, uint16_t *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_rne(x[i]);
}

// ---- mean-pooling of the masks ------------------------------------------------------------

// out [B][nm][nz/2][ny/2][nx/2] = (number of set voxels of mask m0 + c in the
// 2x2x2 block) / 8 for output channel c.
template <class T>
__global__ void meanpool_db_kernel(const uint32_t *__restrict__ planes, int Wp, int nxw, int ny,
                                   int nz, int nx, const int32_t *__restrict__ idx, int B, int m0,
                                   int nm, T *__restrict__ out)
{
    const int X = nx / 2, Y = ny / 2, Z = nz / 2;
    const int64_t per = (int64_t)nm * Z * Y * X;
    const int64_t total = per * B;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t / per);
        int64_t r = t - (int64_t)b * per;
        const int x = (int)(r % X);
        r /= X;
        const int y = (int)(r % Y);
        r /= Y;
        const int z = (int)(r % Z);
        const int m = m0 + (int)(r / Z);
        const uint32_t *pl = planes + (int64_t)idx[b] * 2 * Wp + (int64_t)m * Wp;
        const int wx = (2 * x) >> 5, bit = (2 * x) & 31;
        int c = 0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const uint32_t wv = pl[((int64_t)(2 * z + dz) * ny + (2 * y + dy)) * nxw + wx];
                c += __builtin_popcount((wv >> bit) & 3u);
            }
        out[t] = (T)c * T(0.125);
    }
}

template <class T>
__global__ void meanpool_labels_kernel(const uint8_t *__restrict__ lab, int B, int nx, int ny,
                                       int nz, int m0, int nm, T *__restrict__ out)
{
    const int X = nx / 2, Y = ny / 2, Z = nz / 2;
    const int64_t per = (int64_t)nm * Z * Y * X;
    const int64_t total = per * B;
    const int64_t V = (int64_t)nx * ny * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t / per);
        int64_t r = t - (int64_t)b * per;
        const int x = (int)(r % X);
        r /= X;
        const int y = (int)(r % Y);
        r /= Y;
        const int z = (int)(r % Z);
        const int m = m0 + (int)(r / Z);
        const uint8_t *l = lab + (int64_t)b * V;
        int c = 0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
                    c += (l[((int64_t)(2 * z + dz) * ny + (2 * y + dy)) * nx + 2 * x + dx] >> m) & 1;
        out[t] = (T)c * T(0.125);
    }
}

// Fast paths of the two pooling kernels above (same results): a thread reads the
// four 2-row slabs of a 2x2x2 block row with wide loads and writes 8 (labels) or
// 16 (packed masks) consecutive outputs per channel.
//
// Labels: nx % 16 == 0. Thread = (b, z, y, group of 8 output x = 16 input bytes per row).
template <class T>
__global__ void __launch_bounds__(256) meanpool_labels_fast_kernel(const uint8_t *__restrict__ lab,
                                                                   int B, int nx, int ny, int nz,
                                                                   int m0, int nm,
                                                                   T *__restrict__ out)
{
    const int X = nx / 2, Y = ny / 2, Z = nz / 2, G = X / 8;
    const int64_t total = (int64_t)B * Z * Y * G;
    const int64_t V = (int64_t)nx * ny * nz;
    const int64_t per = (int64_t)Z * Y * X;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(t % G);
        int64_t r = t / G;
        const int y = (int)(r % Y);
        r /= Y;
        const int z = (int)(r % Z);
        const int b = (int)(r / Z);
        // Per mask: SWAR byte sums over the 4 rows (each byte counts 0..4).
        uint32_t f[4] = {0u, 0u, 0u, 0u}, h[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const u32x4 v = *reinterpret_cast<const u32x4 *>(
                    lab + b * V + ((int64_t)(2 * z + dz) * ny + (2 * y + dy)) * nx + 16 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    f[e] += v[e] & 0x01010101u;
                    h[e] += (v[e] >> 1) & 0x01010101u;
                }
            }
        const int64_t o = ((int64_t)b * nm) * per + ((int64_t)z * Y + y) * X + 8 * g;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int m = m0 + c;
            if (c >= nm) break;
            const uint32_t *s = m == 0 ? f : h;
            T v8[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t w = s[e];
                v8[2 * e] = (T)((w & 0xffu) + ((w >> 8) & 0xffu)) * T(0.125);
                v8[2 * e + 1] = (T)(((w >> 16) & 0xffu) + (w >> 24)) * T(0.125);
            }
            T *dst = out + o + (int64_t)c * per;
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[e] = v8[e];
        }
    }
}

// Packed masks: nx % 32 == 0. Thread = (b, mask, z, y, word of 32 input x = 16 outputs).
// First encoder layer straight from query labels: pooled = 2x2x2 mean of the
// masks (values k/8, exact in bfloat16), then the stride-2 convolution on the
// BF16 matrix cores (each product of two bfloat16 values is exact in FP32; the
// sum is FP32). A block takes 2 x 4 x 32 output voxels of one sample: it pools
// the 5 x 9 x 65 patch of pooled voxels it reads into LDS, one 32-bit word per
// pooled voxel (channel 0 in the low half, channel 1 in the high half), rows of
// kPlRow words with pooled x = 2 ow0 - 1 + c at column c + 3. The reduction
// index k < 64 of the two 16 x 16 x 32 products is tap 16 s + k / 2 (s = step),
// channel k % 2, so a lane's eight values of one step are four whole words.
// Each wave owns four tiles of 16 voxels along x; output channels are the 16
// rows (Co <= 16). XCD-aware: the tiles one XCD receives are neighbours, so the
// pooled halo rows they share come from its L2.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
constexpr int kPlRow = 68;


__device__ __forceinline__ uint32_t pooled_word(uint32_t f, uint32_t h, int e)
{
    // Byte pair e of the row sums: counts of the two label columns of one pooled x.
    const uint32_t cf = ((f >> (16 * e)) & 0xffu) + ((f >> (16 * e + 8)) & 0xffu);
    const uint32_t ch = ((h >> (16 * e)) & 0xffu) + ((h >> (16 * e + 8)) & 0xffu);
    const uint32_t bf = __float_as_uint((float)cf * 0.125f) >> 16;   // exact: k/8
    const uint32_t bh = __float_as_uint((float)ch * 0.125f) >> 16;
    return bf | (bh << 16);
}

// The pooled word of counts cf, ch (0..8 set voxels of the two masks in a 2x2x2 block).
__device__ __forceinline__ uint32_t pooled_counts(uint32_t cf, uint32_t ch)
{
    const uint32_t bf = __float_as_uint((float)cf * 0.125f) >> 16;   // exact: k/8
    const uint32_t bh = __float_as_uint((float)ch * 0.125f) >> 16;
    return bf | (bh << 16);
}

// 16 mask bits (8 pairs of x-neighbours) -> the pair counts, 4 bits per pair:
// pair p in bits 4p .. 4p + 3 (room for the sum over four rows, at most 8).
__device__ __forceinline__ uint32_t pair_counts4(uint32_t x16)
{
    uint32_t t = (x16 & 0x5555u) + ((x16 >> 1) & 0x5555u);   // 2-bit pair counts
    t = (t | (t << 8)) & 0x00ff00ffu;
    t = (t | (t << 4)) & 0x0f0f0f0fu;
    return (t | (t << 2)) & 0x33333333u;
}

// The first layer's weights as this lane's A operands (row co = j, eight k from 8 g per
// step), its four biases (rows 4 g .. + 3) and the LDS word of each of its four taps per
// step for the wave's first 16 voxels (tap >= 27: weight zero, any word). Wave w owns the
// tile's voxels 64 w .. + 63: output z = w / 2, y = 2 (w % 2) + m / 2 and x = 16 (m % 2) + j
// for its four products m, so voxels m sit at the compile-time offsets of tile_moff.
__device__ __forceinline__ void first_layer_setup(const uint16_t *__restrict__ Wt,
                                                  const float *__restrict__ bias, int Ci, int Co,
                                                  int wave, int g, int j, bf16x8 (&a)[2],
                                                  float (&bco)[4], int (&ad)[2][4])
{
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int tap = 16 * st + 4 * g + (e >> 1), c = e & 1;
            uint16_t bits = 0;
            if (j < Co && tap < 27 && c < Ci) bits = Wt[((int64_t)j * Ci + c) * 27 + tap];
            a[st][e] = __builtin_bit_cast(__bf16, bits);
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) bco[r] = (bias && 4 * g + r < Co) ? bias[4 * g + r] : 0.f;
    const int base = (18 * (wave >> 1) + 4 * (wave & 1)) * kPlRow + 2 * j + 3;
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tap = 16 * st + 4 * g + i;
            ad[st][i] = base + (tap < 27 ? ((tap / 9) * 9 + (tap / 3) % 3) * kPlRow + tap % 3 : 0);
        }
}

// LDS offset of product m's voxels from the wave's first ones: one output y row is two
// pooled rows, 16 output x are 32 pooled x.
__device__ __forceinline__ constexpr int tile_moff(int m) { return (m >> 1) * 2 * kPlRow + (m & 1) * 32; }

// One tile of the first layer from its pooled patch in LDS (pl, laid out as above): the
// 2 x 4 x 32 output voxels at (od0, oh0, ow0) of sample b, two 16 x 16 x 32 products per
// 16 voxels, then bias, ReLU and the store.
template <bool OUTBF>
__device__ __forceinline__ void first_layer_tile(const uint32_t *pl, const bf16x8 (&a)[2],
                                                 const float (&bco)[4], const int (&ad)[2][4],
                                                 int wave, int g, int j, int od0, int oh0,
                                                 int ow0, int OD, int OH, int OW, int b, int Co,
                                                 int relu, void *__restrict__ Yv)
{
    const int64_t osp = (int64_t)OD * OH * OW;
    const int oz = od0 + (wave >> 1), oy0 = oh0 + 2 * (wave & 1);
    // Output index of product 0's voxel; product m adds (m % 2) 16 + (m / 2) OW.
    const int64_t o0 = ((int64_t)oz * OH + oy0) * OW + ow0 + j;
    const float lo = relu ? 0.f : -INFINITY;       // values below lo become 0 (ReLU)
    uint16_t *Yb = static_cast<uint16_t *>(Yv) + ((int64_t)b * osp + o0) * Co + 4 * g;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const u32x4 bw = {pl[ad[st][0] + tile_moff(m)], pl[ad[st][1] + tile_moff(m)],
                              pl[ad[st][2] + tile_moff(m)], pl[ad[st][3] + tile_moff(m)]};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[st], __builtin_bit_cast(bf16x8, bw),
                                                          acc, 0, 0, 0);
        }
        if (oz >= OD || oy0 + (m >> 1) >= OH) continue;
        const int64_t o = o0 + (m & 1) * 16 + (m >> 1) * OW;
        float yv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            yv[r] = acc[r] + bco[r];
            yv[r] = yv[r] < lo ? 0.f : yv[r];
        }
        if constexpr (OUTBF) {
            if (4 * g < Co)                        // four channels, one 8-byte store
                *reinterpret_cast<u32x2 *>(Yb + ((m & 1) * 16 + (m >> 1) * OW) * Co) =
                    (u32x2){bf16x2_rne(yv[0], yv[1]), bf16x2_rne(yv[2], yv[3])};
        } else {
            float *Y = static_cast<float *>(Yv);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * g + r < Co) Y[((int64_t)b * Co + 4 * g + r) * osp + o] = yv[r];
        }
    }
}

// PLANES: the masks come packed (LSB-first uint32 words, x fastest; plane 0
// FLAIR, plane 1 T1Gd, sample_words = 2 Wp per sample, sample b at
// planes + (idx ? idx[b] : b) * sample_words) instead of as label bytes: a
// pooled row is 4 x 16 bits per mask instead of 4 x 16 bytes.
//
// OUTBF: Y is bfloat16 channels-last [B][nz/4][ny/4][nx/4][Co] (round to nearest even of the
// FP32 result; Co % 4 == 0), the activation layout of the BF16 forward below; otherwise float
// [B][Co][nz/4][ny/4][nx/4].
template <bool PLANES, bool OUTBF>
__global__ void __launch_bounds__(256) pool_conv_labels_kernel(const uint8_t *__restrict__ lab,
                                                               const uint32_t *__restrict__ planes,
                                                               int64_t sample_words,
                                                               const int32_t *__restrict__ idx,
                                                               int nx, int ny, int nz, int mask,
                                                               int Ci, int Co, int npb,
                                                               const uint16_t *__restrict__ Wt,
                                                               const float *__restrict__ bias,
                                                               int relu, void *__restrict__ Yv)
{
    __shared__ __attribute__((aligned(16))) uint32_t pl[45 * kPlRow];
    // PLANES: the raw mask words of the patch, [pooled row][label row q][mask][halo word,
    // 4 words of 128 label x], loaded whole (one 16-byte load per row and mask).
    __shared__ __attribute__((aligned(16))) uint32_t rb[PLANES ? 45 * 8 * 5 : 1];
    const int PZ = nz / 2, PY = ny / 2;
    const int OD = nz / 4, OH = ny / 4, OW = nx / 4;
    const int tw_n = OW / 32, th_n = (OH + 3) / 4, td_n = (OD + 1) / 2;
    const int T = tw_n * th_n * td_n;
    // This block's npb consecutive tiles; with T % (8 npb) == 0 the tiles one XCD
    // receives (blocks x, x + 8, ...) form one contiguous run.
    int t0 = blockIdx.x * npb;
    if (T % (8 * npb) == 0) t0 = (blockIdx.x % 8) * (T / 8) + (blockIdx.x / 8) * npb;
    const int b = blockIdx.y;
    const uint8_t *L = PLANES ? nullptr : lab + (int64_t)b * nz * ny * nx;
    const uint32_t *P = PLANES ? planes + (int64_t)(idx ? idx[b] : b) * sample_words : nullptr;
    const int64_t Wp = sample_words / 2;
    const int nxw = nx / 32;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
    bf16x8 a[2];
    float bco[4];
    int ad[2][4];
    first_layer_setup(Wt, bias, Ci, Co, wave, g, j, a, bco, ad);
    // Pooling items: 45 pooled rows x 8 groups of 8 pooled x (16 label bytes per label
    // row), plus one halo column per row (pooled x = 2 ow0 - 1): 405, at most two per
    // thread. The labels of the next tile are loaded while the current one is computed.
    bool halo[2];
    int row[2], seg[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int it = tid + 256 * u;
        halo[u] = it >= 360;
        row[u] = halo[u] ? it - 360 : it >> 3;
        seg[u] = it & 7;
    }
    u32x4 v[2][4];             // label bytes: 16 per row
    // PLANES: raw row i < 360 (pooled row i / 8, label row q = (i / 2) % 4, mask i % 2) is
    // the 4 words of label x 4 ow0 .. + 127 and the word before (the halo); thread tid
    // loads rows tid and tid + 256.
    u32x4 rw[2] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
    uint32_t rh[2] = {0u, 0u};
    auto load_raw = [&](int t) {
        const int twi = t % tw_n, thi = (t / tw_n) % th_n, tdi = t / (tw_n * th_n);
        const int od0 = 2 * tdi, oh0 = 4 * thi, ow0 = 32 * twi;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = tid + 256 * u, rrow = i >> 3, rq = (i >> 1) & 3, rm = i & 1;
            const int Z = 2 * od0 - 1 + rrow / 9, Yp = 2 * oh0 - 1 + rrow % 9;
            rw[u] = (u32x4){0u, 0u, 0u, 0u};
            rh[u] = 0u;
            if (i < 360 && Z >= 0 && Z < PZ && Yp >= 0 && Yp < PY) {
                const int64_t w = ((int64_t)(2 * Z + (rq >> 1)) * ny + 2 * Yp + (rq & 1)) * nxw +
                                  (4 * ow0) / 32 + rm * Wp;
                rw[u] = *reinterpret_cast<const u32x4 *>(P + w);
                if (ow0 > 0) rh[u] = P[w - 1];
            }
        }
    };
    auto load = [&](int t) {
        if (PLANES) {
            load_raw(t);
            return;
        }
        const int twi = t % tw_n, thi = (t / tw_n) % th_n, tdi = t / (tw_n * th_n);
        const int od0 = 2 * tdi, oh0 = 4 * thi, ow0 = 32 * twi;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int Z = 2 * od0 - 1 + row[u] / 9, Yp = 2 * oh0 - 1 + row[u] % 9;
            const bool in = tid + 256 * u < 405 && Z >= 0 && Z < PZ && Yp >= 0 && Yp < PY &&
                            !(halo[u] && ow0 == 0);
            const uint8_t *r0 = L + ((int64_t)(2 * Z) * ny + 2 * Yp) * nx;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint8_t *r = r0 + ((int64_t)(q >> 1) * ny + (q & 1)) * nx;
                v[u][q] = (u32x4){0u, 0u, 0u, 0u};
                if (in && !halo[u])
                    v[u][q] = *reinterpret_cast<const u32x4 *>(r + 4 * ow0 + 16 * seg[u]);
                else if (in)
                    v[u][q].x = *reinterpret_cast<const uint16_t *>(r + 4 * ow0 - 2);
            }
        }
    };
    load(t0);
    for (int n = 0; n < npb; ++n) {
        const int t = t0 + n;
        if (t >= T) break;                         // uniform over the block
        if (PLANES) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (tid + 256 * u >= 360) break;
                uint32_t *d = &rb[(tid + 256 * u) * 5];
                d[0] = rh[u];
                d[1] = rw[u].x;
                d[2] = rw[u].y;
                d[3] = rw[u].z;
                d[4] = rw[u].w;
            }
            __syncthreads();
            if (n + 1 < npb && t + 1 < T) load_raw(t + 1);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (tid + 256 * u >= 405) break;
            if (PLANES) {
                // Item (row, seg): label x 16 seg .. + 15 of the patch = bits 16 (seg % 2)
                // .. + 15 of raw word 1 + seg / 2; the halo's two columns are bits 30, 31
                // of the word before.
                const int wi = halo[u] ? 0 : 1 + (seg[u] >> 1);
                const int sh = halo[u] ? 30 : 16 * (seg[u] & 1);
                const uint32_t fm = halo[u] ? 3u : 0xffffu;
                uint32_t F = 0u, H = 0u;     // counts of pooled x 0..7, 4 bits each
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t *src = &rb[(row[u] * 8 + q * 2) * 5];
                    F += pair_counts4((src[wi] >> sh) & fm);
                    H += pair_counts4((src[5 + wi] >> sh) & fm);
                }
                if (Ci == 1) {               // one mask: channel 0, channel 1 zero
                    if (mask == 1) F = H;
                    H = 0u;
                }
                if (!halo[u]) {
                    uint32_t w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) w[e] = pooled_counts((F >> (4 * e)) & 15u, (H >> (4 * e)) & 15u);
                    u32x4 *dst = reinterpret_cast<u32x4 *>(&pl[row[u] * kPlRow + 4 + 8 * seg[u]]);
                    dst[0] = (u32x4){w[0], w[1], w[2], w[3]};
                    dst[1] = (u32x4){w[4], w[5], w[6], w[7]};
                } else {
                    pl[row[u] * kPlRow + 3] = pooled_counts(F & 15u, H & 15u);
                }
                continue;
            }
            uint32_t f[4] = {0u, 0u, 0u, 0u}, h[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    f[e] += v[u][q][e] & 0x01010101u;
                    h[e] += (v[u][q][e] >> 1) & 0x01010101u;
                }
            if (Ci == 1) {       // one mask: it goes to channel 0, channel 1 stays zero
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (mask == 1) f[e] = h[e];
                    h[e] = 0u;
                }
            }
            if (!halo[u]) {
                uint32_t w[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    w[2 * e] = pooled_word(f[e], h[e], 0);
                    w[2 * e + 1] = pooled_word(f[e], h[e], 1);
                }
                u32x4 *dst = reinterpret_cast<u32x4 *>(&pl[row[u] * kPlRow + 4 + 8 * seg[u]]);
                dst[0] = (u32x4){w[0], w[1], w[2], w[3]};
                dst[1] = (u32x4){w[4], w[5], w[6], w[7]};
            } else {
                pl[row[u] * kPlRow + 3] = pooled_word(f[0], h[0], 0);
            }
        }
        __syncthreads();
        if (!PLANES && n + 1 < npb && t + 1 < T) load(t + 1);
        const int twi = t % tw_n, thi = (t / tw_n) % th_n, tdi = t / (tw_n * th_n);
        first_layer_tile<OUTBF>(pl, a, bco, ad, wave, g, j, 2 * tdi, 4 * thi, 32 * twi, OD, OH,
                                OW, b, Co, relu, Yv);
        __syncthreads();                           // the next tile overwrites pl
    }
}

// The first layer from pooled counts instead of labels: C is uint8 [B][nz/2][ny/2][nx/2],
// per 2x2x2 block of label voxels its FLAIR count (0..8) in bits 0..3 and its T1Gd count in
// bits 4..7. The pooled means are the counts / 8, so the LDS words, the products and their
// order are pool_conv_labels_kernel's and Y equals its output bit for bit. A tile's patch is
// 45 pooled rows of 64 counts and the count before each row (the halo): 720 groups of four
// counts and 45 halo counts, three per thread, the next tile's in flight while the current
// one is computed.
__device__ __forceinline__ void count_words(uint32_t cb, int Ci, int mask, uint32_t (&w)[4])
{
    // A count k in 0..8 read as an e4m3 FP8 code is k 2^-9 exactly (codes 1..7 are
    // subnormal, 8 is 2^-6), so the scaled FP8 -> bfloat16 pair conversion with scale 2^6
    // gives k / 8: each count pair (FLAIR, T1Gd), interleaved into byte pairs, becomes one
    // word in one instruction. One mask: it goes to channel 0, channel 1 stays zero.
    uint32_t f = cb & 0x0f0f0f0fu, h = (cb >> 4) & 0x0f0f0f0fu;
    if (Ci == 1) {
        if (mask == 1) f = h;
        h = 0u;
    }
    const uint32_t lo = __builtin_amdgcn_perm(h, f, 0x05010400u);   // f0 h0 f1 h1
    const uint32_t hi = __builtin_amdgcn_perm(h, f, 0x07030602u);   // f2 h2 f3 h3
    w[0] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 64.f, false));
    w[1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 64.f, true));
    w[2] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 64.f, false));
    w[3] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 64.f, true));
}

template <bool OUTBF>
__global__ void __launch_bounds__(256) pool_conv_counts_kernel(const uint8_t *__restrict__ C,
                                                               int nx, int ny, int nz, int mask,
                                                               int Ci, int Co, int npb,
                                                               const uint16_t *__restrict__ Wt,
                                                               const float *__restrict__ bias,
                                                               int relu, void *__restrict__ Yv)
{
    __shared__ __attribute__((aligned(16))) uint32_t pl[45 * kPlRow];
    const int PZ = nz / 2, PY = ny / 2, PX = nx / 2;
    const int OD = nz / 4, OH = ny / 4, OW = nx / 4;
    const int tw_n = OW / 32, th_n = (OH + 3) / 4, td_n = (OD + 1) / 2;
    const int T = tw_n * th_n * td_n;
    int t0 = blockIdx.x * npb;
    if (T % (8 * npb) == 0) t0 = (blockIdx.x % 8) * (T / 8) + (blockIdx.x / 8) * npb;
    const int b = blockIdx.y;
    const uint8_t *Cb = C + (int64_t)b * PZ * PY * PX;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
    bf16x8 a[2];
    float bco[4];
    int ad[2][4];
    first_layer_setup(Wt, bias, Ci, Co, wave, g, j, a, bco, ad);
    // Item it = tid + 256 s: it < 720 is group it % 16 (pooled x 2 ow0 + 4 (it % 16) .. + 3) of
    // patch row it / 16; 720 <= it < 765 is the halo count (pooled x 2 ow0 - 1) of row it - 720,
    // zero at ow0 = 0 like the rows outside the volume. Patch row r is pooled z 2 od0 - 1 + r / 9,
    // pooled y 2 oh0 - 1 + r % 9.
    int rz[3], ry[3], lds[3];
    int64_t roff[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int it = tid + 256 * s;
        const int r = it < 720 ? it >> 4 : min(it - 720, 44);
        rz[s] = r / 9 - 1;
        ry[s] = r % 9 - 1;
        roff[s] = ((int64_t)rz[s] * PY + ry[s]) * PX + (it < 720 ? 4 * (it & 15) : -1);
        lds[s] = r * kPlRow + (it < 720 ? 4 + 4 * (it & 15) : 3);
    }
    uint32_t v[3];
    auto load = [&](int t) {
        const int twi = t % tw_n, thi = (t / tw_n) % th_n, tdi = t / (tw_n * th_n);
        const int z0 = 4 * tdi, y0 = 8 * thi, x0 = 64 * twi;   // pooled corner of the patch + 1
        const int64_t toff = ((int64_t)z0 * PY + y0) * PX + x0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int it = tid + 256 * s, Z = z0 + rz[s], Yp = y0 + ry[s];
            v[s] = 0u;
            if (it < 765 && Z >= 0 && Z < PZ && Yp >= 0 && Yp < PY) {
                if (it < 720) v[s] = *reinterpret_cast<const uint32_t *>(Cb + toff + roff[s]);
                else if (x0 > 0) v[s] = Cb[toff + roff[s]];
            }
        }
    };
    load(t0);
    for (int n = 0; n < npb; ++n) {
        const int t = t0 + n;
        if (t >= T) break;                         // uniform over the block
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int it = tid + 256 * s;
            if (it >= 765) break;
            uint32_t w[4];
            count_words(v[s], Ci, mask, w);
            if (it < 720) *reinterpret_cast<u32x4 *>(&pl[lds[s]]) = (u32x4){w[0], w[1], w[2], w[3]};
            else pl[lds[s]] = w[0];
        }
        __syncthreads();
        if (n + 1 < npb && t + 1 < T) load(t + 1);
        const int twi = t % tw_n, thi = (t / tw_n) % th_n, tdi = t / (tw_n * th_n);
        first_layer_tile<OUTBF>(pl, a, bco, ad, wave, g, j, 2 * tdi, 4 * thi, 32 * twi, OD, OH,
                                OW, b, Co, relu, Yv);
        __syncthreads();                           // the next tile overwrites pl
    }
}

// ---- BF16 forward (inference) -----------------------------------------------------------
//
// The later encoder convolutions with bfloat16 activations. X is channels-last bfloat16
// [B][D][H][W][CI]; Y is channels-last bfloat16 [B][D/2][H/2][W/2][CO] (round to nearest even
// of the FP32 result) or, OUTF32, float [B][CO][D/2][H/2][W/2] (the flatten order of the
// linear head). An implicit GEMM on the BF16 matrix cores,
// Y[co][v] = sum over (tap, ci) of Wtm[co][tap][ci] X[2 v + tap - 1][ci], with the tap-major
// weights of conv_w_tapmajor_kernel (28 taps, the last zero). One 16 x 16 x 32 product takes
// four groups of eight channels: in step s, lane quarter q gives group kg = 4 s + q (tap
// kg / NG, channels 8 (kg % NG) .. + 7); rows are 16 output channels, columns 16 output
// voxels. Each product of two bfloat16 values is exact in FP32; the sums are FP32. A block
// takes a TD x TH x TW box of output voxels of one sample (four waves; a wave owns MV voxel
// tiles and MC channel tiles) and stages the input patch in LDS split by x parity, so the
// taps of consecutive output x read consecutive voxels of one parity. The channel groups of
// a patch voxel are rotated by its row (group g stored at g ^ ((py / 2) % NG)), so the rows
// one voxel tile spans fall on different LDS banks.
template <int CI, int CO, int TD, int TH, int TW, bool OUTF32>
__global__ void __launch_bounds__(256, 4) conv_bf16_kernel(int D, int H, int W, int tiles_h,
                                                           int tiles_w, int T, int npb,
                                                           const uint16_t *__restrict__ X,
                                                           const uint16_t *__restrict__ Wtm,
                                                           const float *__restrict__ bias,
                                                           int relu, void *__restrict__ Yv)
{
    constexpr int NG = CI / 8, S = 7 * NG;
    constexpr int NVT = TD * TH * TW / 16, NCO = CO / 16;
    constexpr int WCO = NCO < 4 ? NCO : 4, WVT = 4 / WCO;
    constexpr int MV = NVT / WVT, MC = NCO / WCO;
    constexpr int PD = 2 * TD + 1, PH = 2 * TH + 1, PW = 2 * TW + 1, HW2 = TW + 1;
    constexpr int NCH = PD * PH * PW * NG;                 // 16-byte chunks of the patch
    constexpr int NIT = (NCH + 255) / 256;
    static_assert(CI % 8 == 0 && (NG & (NG - 1)) == 0 && CO % 16 == 0, "channels");
    static_assert((TD * TH * TW) % 16 == 0 && NVT % WVT == 0 && NCO % WCO == 0, "tile");
    __shared__ __attribute__((aligned(16))) uint16_t xs[PD * PH * 2 * HW2 * CI];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, j = lane & 15;
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int per = (OD / TD) * tiles_h * tiles_w;         // tiles per sample
    // This block's npb consecutive tiles (numbered over all samples, T in all); the next
    // tile's patch is loaded into registers while the current one is multiplied.
    const int t0 = blockIdx.x * npb;
    u32x4 v[NIT];
    auto load = [&](int gt) {
        const int b = gt / per, t = gt - b * per;
        const uint16_t *Xb = X + (int64_t)b * D * H * W * CI;
        const int tw = t % tiles_w, th = (t / tiles_w) % tiles_h, td = t / (tiles_w * tiles_h);
        const int iz0 = 2 * td * TD - 1, iy0 = 2 * th * TH - 1, ix0 = 2 * tw * TW - 1;
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = i * 256 + tid;
            const int g = e % NG, r = e / NG;
            const int px = r % PW, py = (r / PW) % PH, pz = r / (PW * PH);
            const int iz = iz0 + pz, iy = iy0 + py, ix = ix0 + px;
            v[i] = (u32x4){0u, 0u, 0u, 0u};
            if (e < NCH && (unsigned)iz < (unsigned)D && (unsigned)iy < (unsigned)H &&
                (unsigned)ix < (unsigned)W)
                v[i] = *reinterpret_cast<const u32x4 *>(
                    Xb + (((int64_t)iz * H + iy) * W + ix) * CI + 8 * g);
        }
    };
    // The lane's voxel of each of its voxel tiles: the slot of its tap (0, 0, 0) and its
    // output row within the tile (the patch row of tap kh is 2 oy + kh).
    int vslot[MV], vrow[MV];
#pragma unroll
    for (int m = 0; m < MV; ++m) {
        const int vv = (wave / WCO + m * WVT) * 16 + j;
        const int oz = vv / (TH * TW), oy = (vv / TW) % TH, ox = vv % TW;
        vslot[m] = (2 * oz * PH + 2 * oy) * 2 * HW2 + ox;
        vrow[m] = oy;
    }
    const uint16_t *wl = Wtm + (int64_t)((wave % WCO) * 16 + j) * 28 * CI + 8 * q;
    const int64_t osp = (int64_t)OD * OH * OW;
    if (t0 < T) load(t0);
    for (int n = 0; n < npb; ++n) {
        const int gt = t0 + n;
        if (gt >= T) break;                                 // uniform over the block
        const int b = gt / per, t = gt - b * per;
        // The patch into LDS (zeros outside the volume), split by x parity.
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = i * 256 + tid;
            if (e < NCH) {
                const int g = e % NG, r = e / NG;
                const int px = r % PW, py = (r / PW) % PH, pz = r / (PW * PH);
                const int slot = ((pz * PH + py) * 2 + (px & 1)) * HW2 + (px >> 1);
                *reinterpret_cast<u32x4 *>(&xs[slot * CI + 8 * (g ^ ((py >> 1) & (NG - 1)))]) =
                    v[i];
            }
        }
        __syncthreads();
        if (n + 1 < npb && gt + 1 < T) load(gt + 1);
        f32x4 acc[MV][MC];
#pragma unroll
        for (int m = 0; m < MV; ++m)
#pragma unroll
            for (int c = 0; c < MC; ++c) acc[m][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < S; ++st) {
            const int kg = 4 * st + q, tap = kg / NG, g = kg % NG;
            const int tp = tap < 27 ? tap : 0;              // tap 27: zero weights
            const int kd = tp / 9, kh = (tp / 3) % 3, kw = tp % 3;
            const int toff = ((kd * PH + kh) * 2 + (kw & 1)) * HW2 + (kw >> 1);
            bf16x8 a[MC];
#pragma unroll
            for (int c = 0; c < MC; ++c)
                a[c] = *reinterpret_cast<const bf16x8 *>(wl + (int64_t)c * WCO * 16 * 28 * CI +
                                                         32 * st);
#pragma unroll
            for (int m = 0; m < MV; ++m) {
                const int off =
                    (vslot[m] + toff) * CI + 8 * (g ^ ((vrow[m] + (kh >> 1)) & (NG - 1)));
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&xs[off]);
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    acc[m][c] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], bv, acc[m][c], 0, 0, 0);
            }
        }
        const int tw = t % tiles_w, th = (t / tiles_w) % tiles_h, td = t / (tiles_w * tiles_h);
#pragma unroll
        for (int m = 0; m < MV; ++m) {
            const int vv = (wave / WCO + m * WVT) * 16 + j;
            const int oz = td * TD + vv / (TH * TW), oy = th * TH + (vv / TW) % TH;
            const int ox = tw * TW + vv % TW;
            const int64_t o = ((int64_t)oz * OH + oy) * OW + ox;
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const int co0 = (wave % WCO + c * WCO) * 16 + 4 * q;
                float y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    y[r] = acc[m][c][r] + (bias ? bias[co0 + r] : 0.f);
                    if (relu && y[r] < 0.f) y[r] = 0.f;
                }
                if constexpr (OUTF32) {
                    float *Y = static_cast<float *>(Yv);
#pragma unroll
                    for (int r = 0; r < 4; ++r) Y[((int64_t)b * CO + co0 + r) * osp + o] = y[r];
                } else {
                    uint16_t *Y = static_cast<uint16_t *>(Yv);
                    const uint32_t lo =
                        f32_to_bf16_rne(y[0]) | ((uint32_t)f32_to_bf16_rne(y[1]) << 16);
                    const uint32_t hi =
                        f32_to_bf16_rne(y[2]) | ((uint32_t)f32_to_bf16_rne(y[3]) << 16);
                    *reinterpret_cast<u32x2 *>(&Y[((int64_t)b * osp + o) * CO + co0]) =
                        (u32x2){lo, hi};
                }
            }
        }
        __syncthreads();                                    // the next patch overwrites xs
    }
}

// ---- The first two layers in one pass ---------------------------------------------------
//
// pool_conv_counts_kernel followed by conv_bf16_kernel<8, 16, ...> without the first layer's
// activations leaving the chip. A block owns the 4 x 16 (y, x) second-layer outputs at
// (Y0, X0) of one sample over zc consecutive output slices and walks them in z. Each step loads
// the next four pooled slices into a ring of five (19 rows of 64 counts and the word before
// each row: the 4 x 16 outputs' pooled patch), computes the next two first-layer slices of the
// second layer's patch (9 rows x 33 x) into a ring of three, then the step's output slice.
// Both layers take the operands, sums and roundings of those two kernels, so Y equals
// conv_bf16(pool_conv_counts(C)) bit for bit (a first-layer sum is never -0, so ReLU as a
// maximum gives the same bits); first-layer voxels outside the volume are the second layer's
// zero padding. ReLU after both layers (the encoder's). CI: 2, or 1 (the mask `mask` alone).
constexpr int kC12Rows = 19;                  // pooled rows of a slice patch: 4 x 4 + 3
constexpr int kC12Half = 17;                  // first-layer voxels per row and x parity
constexpr int kC12L1 = 9 * 2 * kC12Half;      // first-layer voxels per slice, 16 bytes each
constexpr int kC12Main = 4 * kC12Rows;        // 16-count groups of a pooled slice

// Pooled item `it` of a load of ns slices: it < 4 ns 19 is group p (16 counts at pooled x
// 4 X0 + 16 p) of row r of slice s; the next 19 ns are the words before the rows (pooled x
// 4 X0 - 4 .. - 1), halo = true.
__device__ __forceinline__ void c12_item(int it, int ns, int &s, int &r, int &p, bool &halo)
{
    halo = it >= ns * kC12Main;
    const int h = it - ns * kC12Main;
    s = halo ? h / kC12Rows : it / kC12Main;
    const int rem = halo ? h - s * kC12Rows : it - s * kC12Main;
    r = halo ? rem : rem >> 2;
    p = halo ? 4 : rem & 3;
}

template <int CI>
__global__ void __launch_bounds__(256, 4) counts_conv12_kernel(
    const uint8_t *__restrict__ C, int nx, int ny, int nz, int mask, int zc, int units,
    const uint16_t *__restrict__ Wt1, const float *__restrict__ b1,
    const uint16_t *__restrict__ Wtm2, const float *__restrict__ b2, uint16_t *__restrict__ Y)
{
    __shared__ __attribute__((aligned(16))) uint32_t pool[5 * kC12Rows * kPlRow];
    __shared__ __attribute__((aligned(16))) uint16_t l1[3 * kC12L1 * 8];
    const int PY = ny / 2, PX = nx / 2;
    const int OD2 = nz / 8, OH2 = ny / 8, OW2 = nx / 8;
    const int tx_n = OW2 / 16, ty_n = OH2 / 4, zc_n = OD2 / zc;
    // Unit u: x tile fastest, then y tile, z chunk, sample. With units % 8 == 0 the units one
    // XCD receives (blocks x, x + 8, ...) are one contiguous run, so the neighbours that share
    // pooled halo rows read them through one L2.
    int u = blockIdx.x;
    if (units % 8 == 0) u = (blockIdx.x % 8) * (units / 8) + blockIdx.x / 8;
    const int tx = u % tx_n, ty = (u / tx_n) % ty_n, zi = (u / (tx_n * ty_n)) % zc_n;
    const int b = u / (tx_n * ty_n * zc_n);
    const int X0 = 16 * tx, Y0 = 4 * ty, oz0 = zi * zc;
    const int64_t slice = (int64_t)PY * PX;
    const uint8_t *Cb = C + (int64_t)b * (nz / 2) * slice + 4 * X0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;

    // First layer: this lane's weights and biases (first_layer_setup's layout), and per tap
    // of its two products the pooled slice (kd) and the offset within the slice.
    bf16x8 a1[2];
    float bc1[4];
    {
        int unused[2][4];
        first_layer_setup(Wt1, b1, CI, 8, 0, g, j, a1, bc1, unused);
    }
    int kd1[2][4], to1[2][4];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tap = 16 * st + 4 * g + i;   // >= 27: weight zero, any written word
            kd1[st][i] = tap < 27 ? tap / 9 : 0;
            to1[st][i] = tap < 27 ? ((tap / 3) % 3) * kPlRow + tap % 3 : 0;
        }
    // Second layer: weights (conv_bf16_kernel's tap-major layout; lane quarter g is the
    // k group), biases, and per product step the first-layer slice (kd) and voxel of the
    // lane's output voxel (row wave, x j).
    bf16x8 a2[7];
    int kd2[7], vo2[7];
#pragma unroll
    for (int st = 0; st < 7; ++st) {
        a2[st] = *reinterpret_cast<const bf16x8 *>(Wtm2 + j * 28 * 8 + 8 * g + 32 * st);
        const int tap = 4 * st + g, tp = tap < 27 ? tap : 0;
        const int kd = tp / 9, kh = (tp / 3) % 3, kw = tp % 3;
        kd2[st] = kd;
        vo2[st] = ((2 * wave + kh) * 2 + (kw & 1)) * kC12Half + j + (kw >> 1);
    }
    float bc2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bc2[r] = b2 ? b2[4 * g + r] : 0.f;

    // The pooled items of the four-slice loads, two per thread: per item its slice, the
    // offset of its counts from slice pzf's row 4 Y0 - 3 (pooled y checked per load) and its
    // LDS word within the slot. At X0 = 0 the words before the rows are zero, written once.
    const int nit = 4 * kC12Main + (X0 > 0 ? 4 * kC12Rows : 0);
    int is[2], iy[2], ig[2], il[2];
    bool ih[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int s, r, p;
        bool halo;
        c12_item(tid + 256 * k, 4, s, r, p, halo);
        is[k] = s;
        iy[k] = 4 * Y0 - 3 + r;
        ig[k] = (int)(s * slice) + iy[k] * PX + (halo ? -4 : 16 * p);
        il[k] = r * kPlRow + (halo ? 0 : 4 + 16 * p);
        ih[k] = halo;
    }
    u32x4 v[2];
    auto load4 = [&](int pzf) {
        const uint8_t *base = Cb + (int64_t)pzf * slice;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            v[k] = (u32x4){0u, 0u, 0u, 0u};
            if (tid + 256 * k < nit && iy[k] >= 0 && iy[k] < PY) {
                if (!ih[k]) v[k] = *reinterpret_cast<const u32x4 *>(base + ig[k]);
                else v[k].x = *reinterpret_cast<const uint32_t *>(base + ig[k]);
            }
        }
    };
    auto words = [&](uint32_t cb, uint32_t *d) {
        uint32_t w[4];
        count_words(cb, CI, mask, w);
        *reinterpret_cast<u32x4 *>(d) = (u32x4){w[0], w[1], w[2], w[3]};
    };
    auto store4 = [&](int pzf) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (tid + 256 * k < nit) {
                uint32_t *d = pool + ((pzf + is[k] + 5) % 5) * kC12Rows * kPlRow + il[k];
                if (!ih[k]) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) words(v[k][e], d + 4 * e);
                } else {
                    words(v[k].x, d);
                }
            }
        }
    };

    // One first-layer slice z1: wave w takes the x half w % 2 of the rows r1 = p, p + 2, ...
    // (p = (w / 2) ^ s, so two slices give every wave nine columns of 16 voxels); with
    // X0 > 0 wave 2 + s also takes the column x = 2 X0 - 1 of the nine rows (lane j = row).
    auto l1_slice = [&](int z1, int s) {
        int sb[3];
#pragma unroll
        for (int kd = 0; kd < 3; ++kd) sb[kd] = ((2 * z1 - 1 + kd + 5) % 5) * kC12Rows * kPlRow;
        const int lsb = ((z1 + 3) % 3) * kC12L1;
        const int p = (wave >> 1) ^ s, h = wave & 1;
        const bool zin = z1 >= 0;
        int o[2][4];
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o[st][i] = (kd1[st][i] == 0 ? sb[0] : kd1[st][i] == 1 ? sb[1] : sb[2]) +
                           to1[st][i] + 2 * p * kPlRow + 32 * h + 2 * j + 3;
        // First-layer voxel x = 2 X0 + 16 h + j is patch column c1 = 1 + 16 h + j.
        const int sl = lsb + p * 2 * kC12Half + ((1 + j) & 1) * kC12Half + 8 * h + ((1 + j) >> 1);
        auto product = [&](int k) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const u32x4 bw = {pool[o[st][0] + 4 * k * kPlRow], pool[o[st][1] + 4 * k * kPlRow],
                                  pool[o[st][2] + 4 * k * kPlRow], pool[o[st][3] + 4 * k * kPlRow]};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[st], __builtin_bit_cast(bf16x8, bw),
                                                              acc, 0, 0, 0);
            }
            return acc;
        };
        // Bias, ReLU, bfloat16 of a column's channels (lanes 0..31); zero for a row r1 = p + 2 k
        // outside the volume (y = 2 Y0 - 1 + r1 < 0 only for r1 = 0, Y0 = 0) or a slice below it.
        auto finish = [&](f32x4 acc, bool inside) {
            float y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = fmaxf(acc[r] + bc1[r], 0.f);
            const uint32_t m = inside ? 0xffffffffu : 0u;
            return (u32x2){bf16x2_rne(y[0], y[1]) & m, bf16x2_rne(y[2], y[3]) & m};
        };
        auto in_vol = [&](int k) { return zin && (p + k > 0 || Y0 > 0); };
        // Columns k, k + 1 in one store: lanes 0..31 (channels 0..7) of column k + 1 go to the
        // unused lanes 32..63 of column k, which then store to column k + 1's slots.
        const int pst = (sl + (g >= 2 ? 4 * kC12Half : 0)) * 8 + 4 * (g & 1);
#pragma unroll
        for (int k = 0; k < 4; k += 2) {
            const u32x2 e0 = finish(product(k), in_vol(k)), e1 = finish(product(k + 1), in_vol(k + 1));
            const u32x2 c = {__builtin_amdgcn_permlane32_swap(e0.x, e1.x, false, false)[0],
                             __builtin_amdgcn_permlane32_swap(e0.y, e1.y, false, false)[0]};
            *reinterpret_cast<u32x2 *>(&l1[pst + 4 * k * kC12Half * 8]) = c;
        }
        if (!p) {                                  // even rows: r1 = 8 as well
            const u32x2 e = finish(product(4), in_vol(4));
            if (g < 2) *reinterpret_cast<u32x2 *>(&l1[(sl + 16 * kC12Half) * 8 + 4 * g]) = e;
        }
        if (X0 > 0 && wave == 2 + s) {
            const int r1 = j < 9 ? j : 8;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                int w4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    w4[i] = (kd1[st][i] == 0 ? sb[0] : kd1[st][i] == 1 ? sb[1] : sb[2]) + to1[st][i] +
                            2 * r1 * kPlRow + 1;
                const u32x4 bw = {pool[w4[0]], pool[w4[1]], pool[w4[2]], pool[w4[3]]};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[st], __builtin_bit_cast(bf16x8, bw),
                                                              acc, 0, 0, 0);
            }
            if (j < 9 && g < 2) {
                float y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fmaxf(acc[r] + bc1[r], 0.f);
                const uint32_t m = zin && (r1 > 0 || Y0 > 0) ? 0xffffffffu : 0u;
                *reinterpret_cast<u32x2 *>(&l1[(lsb + r1 * 2 * kC12Half) * 8 + 4 * g]) =
                    (u32x2){bf16x2_rne(y[0], y[1]) & m, bf16x2_rne(y[2], y[3]) & m};
            }
        }
    };

    // At X0 = 0 the column x = -1 of every first-layer slice is padding and the word before
    // every pooled row is zero: both written once, never again.
    if (X0 == 0) {
        if (tid < 27)
            *reinterpret_cast<u32x4 *>(&l1[((tid % 3) * kC12L1 + (tid / 3) * 2 * kC12Half) * 8]) =
                (u32x4){0u, 0u, 0u, 0u};
        else if (tid < 27 + 5 * kC12Rows)
            *reinterpret_cast<u32x4 *>(&pool[(tid - 27) * kPlRow]) = (u32x4){0u, 0u, 0u, 0u};
    }
    // Prologue: the first-layer slice 2 oz0 - 1 from pooled slices 4 oz0 - 3 .. - 1 (zero
    // below the volume), its items computed here.
    {
        const int pzf = 4 * oz0 - 3, n3 = 3 * kC12Main + (X0 > 0 ? 3 * kC12Rows : 0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int it = tid + 256 * k;
            if (it < n3) {
                int s, r, p;
                bool halo;
                c12_item(it, 3, s, r, p, halo);
                const int pz = pzf + s, py = 4 * Y0 - 3 + r;
                uint32_t *d = pool + ((pz + 5) % 5) * kC12Rows * kPlRow + r * kPlRow;
                u32x4 x = {0u, 0u, 0u, 0u};
                if (pz >= 0 && py >= 0 && py < PY) {
                    const uint8_t *row = Cb + pz * slice + (int64_t)py * PX;
                    if (!halo) x = *reinterpret_cast<const u32x4 *>(row + 16 * p);
                    else x.x = *reinterpret_cast<const uint32_t *>(row - 4);
                }
                if (!halo) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) words(x[e], d + 4 + 16 * p + 4 * e);
                } else {
                    words(x.x, d);
                }
            }
        }
    }
    load4(4 * oz0);
    __syncthreads();
    l1_slice(2 * oz0 - 1, 0);
    __syncthreads();
    const int64_t yrow = (int64_t)OH2 * OW2;
    for (int oz = oz0; oz < oz0 + zc; ++oz) {
        store4(4 * oz);
        if (oz + 1 < oz0 + zc) load4(4 * oz + 4);   // in flight during the products
        __syncthreads();
        l1_slice(2 * oz, 0);
        l1_slice(2 * oz + 1, 1);
        __syncthreads();
        // Second layer: output row Y0 + wave, x X0 + j, channels 4 g .. + 3.
        int lb[3];
#pragma unroll
        for (int kd = 0; kd < 3; ++kd) lb[kd] = ((2 * oz - 1 + kd + 3) % 3) * kC12L1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 7; ++st) {
            const int vox = (kd2[st] == 0 ? lb[0] : kd2[st] == 1 ? lb[1] : lb[2]) + vo2[st];
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&l1[vox * 8]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[st], bv, acc, 0, 0, 0);
        }
        float y[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = fmaxf(acc[r] + bc2[r], 0.f);
        const int64_t o = (((int64_t)b * OD2 + oz) * yrow + (int64_t)(Y0 + wave) * OW2 + X0 + j) * 16;
        *reinterpret_cast<u32x2 *>(&Y[o + 4 * g]) = (u32x2){bf16x2_rne(y[0], y[1]), bf16x2_rne(y[2], y[3])};
    }
}

// ---- The third and fourth layers in one pass, per sample ------------------------------------
//
// conv_bf16_kernel<16, 32, ...> (bfloat16 output) followed by conv_bf16_kernel<32, 64, ...>
// (float output) for a 16^3 x 16-channel input: a block per sample streams the input through
// a ring of three z-slices in LDS, computes each 8 x 8 output slice of the third layer into an
// LDS copy of its whole 8^3 x 32 output, then the fourth layer's 4^3 x 64 outputs from it. The
// operands (k = 32 per product: lane quarter g takes tap kg / NG, channels 8 (kg % NG) .. + 7
// with kg = 4 st + g), sums and roundings are those kernels': Y equals theirs bit for bit.
// Zero padding by range checks on the operand reads (no halo stored).
constexpr int kC34In = 16 * 16 * 16;              // one input slice: 16 x 16 voxels x 16 ch (bf16)
constexpr int kC34Mid = 8 * 8 * 8 * 32;           // the third layer's output, bf16

__global__ void __launch_bounds__(512, 1) conv34_kernel(const uint16_t *__restrict__ X,
                                                        const uint16_t *__restrict__ Wtm3,
                                                        const float *__restrict__ b3,
                                                        const uint16_t *__restrict__ Wtm4,
                                                        const float *__restrict__ b4,
                                                        float *__restrict__ Y)
{
    __shared__ __attribute__((aligned(16))) uint16_t ring[3 * kC34In];
    __shared__ __attribute__((aligned(16))) uint16_t mid[kC34Mid];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const uint16_t *Xb = X + (int64_t)b * 16 * kC34In;
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, (u32x4){0u, 0u, 0u, 0u});

    // Two input slices (16 KB) per step, 32 bytes per thread: z = zs, zs + 1.
    u32x4 v[2];
    auto load2 = [&](int zs) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = tid + 512 * u, z = zs + (c >> 9);           // 512 chunks per slice
            v[u] = z < 16 ? *reinterpret_cast<const u32x4 *>(Xb + (int64_t)z * kC34In + 8 * (c & 511))
                          : (u32x4){0u, 0u, 0u, 0u};
        }
    };
    auto store2 = [&](int zs) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = tid + 512 * u, z = zs + (c >> 9);
            *reinterpret_cast<u32x4 *>(&ring[((z + 3) % 3) * kC34In + 8 * (c & 511)]) = v[u];
        }
    };

    // Third layer: wave w owns output rows oy = 2 (w / 2), + 1 (voxel tile of 16: oy = 2 (w / 2)
    // + j / 8, ox = j % 8) and the 16-channel tile w % 2.
    const int oy = 2 * (wave >> 1) + (j >> 3), ox = j & 7, ct = wave & 1;
    const uint16_t *w3 = Wtm3 + (ct * 16 + j) * 28 * 16 + 8 * g;
    float bias3[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bias3[r] = b3 ? b3[ct * 16 + 4 * g + r] : 0.f;

    load2(0);                      // slices 0, 1; slice -1 is padding
    for (int z3 = 0; z3 < 8; ++z3) {
        store2(2 * z3);
        if (z3 + 1 < 8) load2(2 * z3 + 2);   // in flight during the products
        __syncthreads();
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 14; ++st) {
            const int kg = 4 * st + g, tap = kg >> 1, cg = kg & 1;
            const int tp = tap < 27 ? tap : 0;
            const int kd = tp / 9, kh = (tp / 3) % 3, kw = tp % 3;
            const int iz = 2 * z3 - 1 + kd, iy = 2 * oy - 1 + kh, ix = 2 * ox - 1 + kw;
            const bool in = iz >= 0 && iy >= 0 && ix >= 0;            // < 16 always
            const bf16x8 bv = in ? *reinterpret_cast<const bf16x8 *>(
                                       &ring[((iz + 3) % 3) * kC34In + (iy * 16 + ix) * 16 + 8 * cg])
                                 : zero8;
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                *reinterpret_cast<const bf16x8 *>(w3 + 32 * st), bv, acc, 0, 0, 0);
        }
        // Bias, ReLU, bfloat16 into the third layer's output [z][y][x][32].
        {
            float y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                y[r] = acc[r] + bias3[r];
                if (y[r] < 0.f) y[r] = 0.f;
            }
            *reinterpret_cast<u32x2 *>(&mid[((z3 * 8 + oy) * 8 + ox) * 32 + ct * 16 + 4 * g]) =
                (u32x2){bf16x2_rne(y[0], y[1]), bf16x2_rne(y[2], y[3])};
        }
        __syncthreads();           // the next step's slices overwrite the ring
    }

    // Fourth layer: wave w owns output channels 16 (w / 2) .. + 15 and the voxel tiles
    // m = 2 (w % 2), + 1 (tile m: oz = m, oy = j / 4, ox = j % 4).
    f32x4 acc4[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const int c4 = wave >> 1, m0 = 2 * (wave & 1);
    const uint16_t *wl = Wtm4 + (int64_t)(c4 * 16 + j) * 28 * 32 + 8 * g;
    const int py = j >> 2, px = j & 3;
#pragma unroll 4
    for (int st = 0; st < 28; ++st) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(wl + 32 * st);
        const int kg = 4 * st + g, tap = kg >> 2, cg = kg & 3;
        const int tp = tap < 27 ? tap : 0;
        const int kd = tp / 9, kh = (tp / 3) % 3, kw = tp % 3;
        const int iy = 2 * py - 1 + kh, ix = 2 * px - 1 + kw;
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int m = m0 + mm, iz = 2 * m - 1 + kd;
            const bool in = iz >= 0 && iy >= 0 && ix >= 0;             // < 8 always
            const bf16x8 bv = in ? *reinterpret_cast<const bf16x8 *>(
                                       &mid[((iz * 8 + iy) * 8 + ix) * 32 + 8 * cg])
                                 : zero8;
            acc4[mm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc4[mm], 0, 0, 0);
        }
    }
    float *Yb = Y + (int64_t)b * 64 * 64;
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = c4 * 16 + 4 * g + r;
            float y = acc4[mm][r] + (b4 ? b4[co] : 0.f);
            if (y < 0.f) y = 0.f;
            Yb[co * 64 + (m0 + mm) * 16 + j] = y;
        }
}

// Tap-major copy of convolution weights for conv_bf16_kernel: out[co][t][ci] = w[co][ci][t]
// (t < 27; the model's [co][ci][kd][kh][kw] order) and 0 for t = 27.
__global__ void conv_w_tapmajor_kernel(int Co, int Ci, const uint16_t *__restrict__ w,
                                       uint16_t *__restrict__ out)
{
    const int64_t n = (int64_t)Co * 28 * Ci;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(e % Ci), tp = (int)((e / Ci) % 28), co = (int)(e / ((int64_t)28 * Ci));
        out[e] = tp < 27 ? w[((int64_t)co * Ci + ci) * 27 + tp] : (uint16_t)0;
    }
}

template <class T>
__global__ void __launch_bounds__(256) meanpool_db_fast_kernel(const uint32_t *__restrict__ planes,
                                                               int Wp, int nxw, int ny, int nz,
                                                               const int32_t *__restrict__ idx,
                                                               int B, int m0, int nm,
                                                               T *__restrict__ out)
{
    const int X = nxw * 16, Y = ny / 2, Z = nz / 2;
    const int64_t total = (int64_t)B * nm * Z * Y * nxw;
    const int64_t per = (int64_t)Z * Y * X;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int wx = (int)(t % nxw);
        int64_t r = t / nxw;
        const int y = (int)(r % Y);
        r /= Y;
        const int z = (int)(r % Z);
        r /= Z;
        const int c = (int)(r % nm);
        const int b = (int)(r / nm);
        const uint32_t *pl = planes + (int64_t)idx[b] * 2 * Wp + (int64_t)(m0 + c) * Wp;
        // Set bits per 2-bit pair, summed over the 4 rows in 4-bit fields (0..8):
        // even pairs in qe, odd pairs in qo.
        uint32_t qe = 0, qo = 0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const uint32_t w = pl[((int64_t)(2 * z + dz) * ny + (2 * y + dy)) * nxw + wx];
                const uint32_t p = (w & 0x55555555u) + ((w >> 1) & 0x55555555u);
                qe += p & 0x33333333u;
                qo += (p >> 2) & 0x33333333u;
            }
        T *dst = out + ((int64_t)b * nm + c) * per + ((int64_t)z * Y + y) * X + 16 * wx;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            dst[2 * j] = (T)((qe >> (4 * j)) & 15u) * T(0.125);
            dst[2 * j + 1] = (T)((qo >> (4 * j)) & 15u) * T(0.125);
        }
    }
}

}  // namespace tdb

// ---- C ABI ----------------------------------------------------------------------------------

using namespace tdb;

namespace {

unsigned grid1(int64_t n, int64_t cap = 4096)
{
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

bool conv_dims_ok(int B, int Ci, int Co, int D, int H, int W)
{
    return B > 0 && Ci > 0 && Co > 0 && D >= 2 && H >= 2 && W >= 2 && !(D & 1) && !(H & 1) &&
           !(W & 1) && B <= 65535 && Ci <= 65535 && Co <= 65535 &&
           (int64_t)D * H * W < ((int64_t)1 << 31);
}

int dtype_pair(int dtype, int wdtype)
{
    if (dtype == NN_F32 && wdtype == NN_BF16) return 0;
    if (dtype == NN_F32 && wdtype == NN_F32) return 1;
    if (dtype == NN_F64 && wdtype == NN_F64) return 2;
    return -1;
}

int launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tdb_set_error(DB_EHIP, "%s: %s", what, hipGetErrorString(e));
    return DB_OK;
}

// Matrix-core forward for float activations: picks the voxel box from the output
// width; a block takes npb tiles of one sample (fewer blocks than tiles keeps the
// loads of the next stage in flight). Returns 1 when the shape is not covered (the
// caller then takes the vector kernel).
template <class WT, int TD, int TH, int TW, int MT>
int conv_mfma_launch(int B, int Ci, int Co, int D, int H, int W, const void *X,
                            const void *Wt, const void *bias, int relu, void *Y, hipStream_t s)
{
    const int nt = (Co + 15) / 16;
    const int OD = D / 2, OH = H / 2, OW = W / 2;
    const int th = (OH + TH - 1) / TH, tw = (OW + TW - 1) / TW;
    const int T = ((OD + TD - 1) / TD) * th * tw;
    const int npb = T >= 64 ? 4 : (T >= 16 ? 2 : 1);
    const dim3 grid((unsigned)((T + npb - 1) / npb), (unsigned)B);
    // All weights in LDS at once when they fit (ConvTile::WALL floats).
    const bool wall = (int64_t)nt * 16 * (27 * Ci + 1) <= 4096;
#define TDB_CONV_MFMA(NT_)                                                                         \
    do {                                                                                           \
        if (wall)                                                                                  \
            hipLaunchKernelGGL((conv_mfma_kernel<WT, TD, TH, TW, MT, NT_, true>), grid, dim3(256), \
                               0, s, Ci, Co, D, H, W, th, tw, T, npb, (const float *)X,            \
                               (const WT *)Wt, (const float *)bias, relu, (float *)Y);             \
        else                                                                                       \
            hipLaunchKernelGGL((conv_mfma_kernel<WT, TD, TH, TW, MT, NT_, false>), grid,           \
                               dim3(256), 0, s, Ci, Co, D, H, W, th, tw, T, npb,                   \
                               (const float *)X, (const WT *)Wt, (const float *)bias, relu,        \
                               (float *)Y);                                                        \
    } while (0)
    switch (nt) {
    case 1: TDB_CONV_MFMA(1); break;
    case 2: TDB_CONV_MFMA(2); break;
    case 3: TDB_CONV_MFMA(3); break;
    default: TDB_CONV_MFMA(4); break;
    }
#undef TDB_CONV_MFMA
    return launched("nn_conv3d_s2_fwd");
}

template <class WT>
int conv_mfma_shape(int B, int Ci, int Co, int D, int H, int W, const void *X,
                           const void *Wt, const void *bias, int relu, void *Y, hipStream_t s)
{
    const int OW = W / 2;
    if (OW >= 16) return conv_mfma_launch<WT, 2, 4, 16, 2>(B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s);
    if (OW >= 8) return conv_mfma_launch<WT, 4, 4, 8, 2>(B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s);
    return conv_mfma_launch<WT, 4, 4, 4, 1>(B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s);
}

int conv_fwd_mfma(bool bf16w, int B, int Ci, int Co, int D, int H, int W, const void *X,
                         const void *Wt, const void *bias, int relu, void *Y, hipStream_t s)
{
    return bf16w ? conv_mfma_shape<uint16_t>(B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s)
                 : conv_mfma_shape<float>(B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s);
}

}  // namespace

extern "C" {

static int meanpool_db(const char *fn, const db_t *db, const int32_t *idx, int B, int m0, int nm,
                       void *out, int dtype, void *stream)
{
    if (!tdb_live(db)) return tdb_set_error(DB_ESTATE, "%s: invalid handle", fn);
    const Geometry &g = db->g;
    if (!idx || !out || B <= 0 || (g.nx & 1) || (g.ny & 1) || (g.nz & 1) ||
        (dtype != NN_F32 && dtype != NN_F64))
        return tdb_set_error(DB_EINVAL, "%s: bad arguments", fn);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t total = (int64_t)B * nm * (g.nz / 2) * (g.ny / 2) * (g.nx / 2);
    if (!(g.nx % 32)) {
        const int64_t tf = total / 16;
        if (dtype == NN_F32)
            hipLaunchKernelGGL(meanpool_db_fast_kernel<float>, dim3(grid1(tf, 65535)), dim3(256), 0, s,
                               db->planes, g.Wp, g.nxw, g.ny, g.nz, idx, B, m0, nm, (float *)out);
        else
            hipLaunchKernelGGL(meanpool_db_fast_kernel<double>, dim3(grid1(tf, 65535)), dim3(256), 0,
                               s, db->planes, g.Wp, g.nxw, g.ny, g.nz, idx, B, m0, nm,
                               (double *)out);
        return launched(fn);
    }
    if (dtype == NN_F32)
        hipLaunchKernelGGL(meanpool_db_kernel<float>, dim3(grid1(total)), dim3(256), 0, s,
                           db->planes, g.Wp, g.nxw, g.ny, g.nz, g.nx, idx, B, m0, nm, (float *)out);
    else
        hipLaunchKernelGGL(meanpool_db_kernel<double>, dim3(grid1(total)), dim3(256), 0, s,
                           db->planes, g.Wp, g.nxw, g.ny, g.nz, g.nx, idx, B, m0, nm, (double *)out);
    return launched(fn);
}

static int meanpool_labels(const char *fn, const uint8_t *labels, int B, int nx, int ny, int nz,
                           int m0, int nm, void *out, int dtype, void *stream)
{
    if (!labels || !out || B <= 0 || nx <= 0 || ny <= 0 || nz <= 0 || (nx & 1) || (ny & 1) ||
        (nz & 1) || (dtype != NN_F32 && dtype != NN_F64))
        return tdb_set_error(DB_EINVAL, "%s: bad arguments", fn);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t total = (int64_t)B * nm * (nz / 2) * (ny / 2) * (nx / 2);
    if (!(nx % 16) && !((uintptr_t)labels % 16)) {
        const int64_t tf = total / nm / 8;
        if (dtype == NN_F32)
            hipLaunchKernelGGL(meanpool_labels_fast_kernel<float>, dim3(grid1(tf, 65535)), dim3(256),
                               0, s, labels, B, nx, ny, nz, m0, nm, (float *)out);
        else
            hipLaunchKernelGGL(meanpool_labels_fast_kernel<double>, dim3(grid1(tf, 65535)),
                               dim3(256), 0, s, labels, B, nx, ny, nz, m0, nm, (double *)out);
        return launched(fn);
    }
    if (dtype == NN_F32)
        hipLaunchKernelGGL(meanpool_labels_kernel<float>, dim3(grid1(total)), dim3(256), 0, s,
                           labels, B, nx, ny, nz, m0, nm, (float *)out);
    else
        hipLaunchKernelGGL(meanpool_labels_kernel<double>, dim3(grid1(total)), dim3(256), 0, s,
                           labels, B, nx, ny, nz, m0, nm, (double *)out);
    return launched(fn);
}

int nn_meanpool_db(const db_t *db, const int32_t *idx, int B, void *out, int dtype, void *stream)
{
    return meanpool_db("nn_meanpool_db", db, idx, B, 0, 2, out, dtype, stream);
}

int nn_meanpool_labels(const uint8_t *labels, int B, int nx, int ny, int nz, void *out, int dtype,
                       void *stream)
{
    return meanpool_labels("nn_meanpool_labels", labels, B, nx, ny, nz, 0, 2, out, dtype, stream);
}

int nn_meanpool_db_mask(const db_t *db, const int32_t *idx, int B, int mask, void *out, int dtype,
                        void *stream)
{
    if (mask != 0 && mask != 1) return tdb_set_error(DB_EINVAL, "nn_meanpool_db_mask: mask %d", mask);
    return meanpool_db("nn_meanpool_db_mask", db, idx, B, mask, 1, out, dtype, stream);
}

int nn_meanpool_labels_mask(const uint8_t *labels, int B, int nx, int ny, int nz, int mask,
                            void *out, int dtype, void *stream)
{
    if (mask != 0 && mask != 1)
        return tdb_set_error(DB_EINVAL, "nn_meanpool_labels_mask: mask %d", mask);
    return meanpool_labels("nn_meanpool_labels_mask", labels, B, nx, ny, nz, mask, 1, out, dtype,
                           stream);
}

int nn_pool_conv_labels(const uint8_t *labels, int B, int nx, int ny, int nz, int mask, int Co,
                        const void *Wt, const float *bias, int relu, float *Y, void *stream)
{
    if (!labels || !Wt || !Y || B <= 0 || B > 65535 || nx <= 0 || ny <= 0 || nz <= 0 ||
        nx % 128 || ny % 4 || nz % 4 || Co <= 0 || Co > 16 || mask < -1 || mask > 1 ||
        (uintptr_t)labels % 16 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_pool_conv_labels: bad arguments");
    const int T = (nx / 128) * ((ny / 4 + 3) / 4) * ((nz / 4 + 1) / 2);
    const int npb = T % 32 == 0 ? 4 : 1;           // tiles per block
    hipLaunchKernelGGL((pool_conv_labels_kernel<false, false>), dim3((unsigned)((T + npb - 1) / npb), (unsigned)B),
                       dim3(256), 0, static_cast<hipStream_t>(stream), labels, nullptr, (int64_t)0,
                       nullptr, nx, ny, nz, mask, mask < 0 ? 2 : 1, Co, npb,
                       static_cast<const uint16_t *>(Wt), bias, relu, Y);
    return launched("nn_pool_conv_labels");
}

int nn_pool_conv_planes(const uint32_t *planes, int64_t sample_words, const int32_t *idx, int B,
                        int nx, int ny, int nz, int mask, int Co, const void *Wt,
                        const float *bias, int relu, float *Y, void *stream)
{
    const int64_t words = (int64_t)nx * ny * nz / 32;
    if (!planes || !Wt || !Y || B <= 0 || B > 65535 || nx <= 0 || ny <= 0 || nz <= 0 ||
        nx % 128 || ny % 4 || nz % 4 || Co <= 0 || Co > 16 || mask < -1 || mask > 1 ||
        sample_words % 2 || sample_words / 2 < words || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_pool_conv_planes: bad arguments");
    const int T = (nx / 128) * ((ny / 4 + 3) / 4) * ((nz / 4 + 1) / 2);
    const int npb = T % 32 == 0 ? 4 : 1;           // tiles per block
    hipLaunchKernelGGL((pool_conv_labels_kernel<true, false>), dim3((unsigned)((T + npb - 1) / npb), (unsigned)B),
                       dim3(256), 0, static_cast<hipStream_t>(stream), nullptr, planes,
                       sample_words, idx, nx, ny, nz, mask, mask < 0 ? 2 : 1, Co, npb,
                       static_cast<const uint16_t *>(Wt), bias, relu, Y);
    return launched("nn_pool_conv_planes");
}

int nn_pool_conv_labels_bf16(const uint8_t *labels, int B, int nx, int ny, int nz, int mask,
                             int Co, const void *Wt, const float *bias, int relu, void *Y,
                             void *stream)
{
    if (!labels || !Wt || !Y || B <= 0 || B > 65535 || nx <= 0 || ny <= 0 || nz <= 0 ||
        nx % 128 || ny % 4 || nz % 4 || Co <= 0 || Co > 16 || Co % 4 || mask < -1 || mask > 1 ||
        (uintptr_t)labels % 16 || (uintptr_t)Y % 8 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_pool_conv_labels_bf16: bad arguments");
    const int T = (nx / 128) * ((ny / 4 + 3) / 4) * ((nz / 4 + 1) / 2);
    const int npb = T % 32 == 0 ? 4 : 1;
    hipLaunchKernelGGL((pool_conv_labels_kernel<false, true>),
                       dim3((unsigned)((T + npb - 1) / npb), (unsigned)B), dim3(256), 0,
                       static_cast<hipStream_t>(stream), labels, nullptr, (int64_t)0, nullptr, nx,
                       ny, nz, mask, mask < 0 ? 2 : 1, Co, npb, static_cast<const uint16_t *>(Wt),
                       bias, relu, Y);
    return launched("nn_pool_conv_labels_bf16");
}

int nn_pool_conv_planes_bf16(const uint32_t *planes, int64_t sample_words, const int32_t *idx,
                             int B, int nx, int ny, int nz, int mask, int Co, const void *Wt,
                             const float *bias, int relu, void *Y, void *stream)
{
    const int64_t words = (int64_t)nx * ny * nz / 32;
    if (!planes || !Wt || !Y || B <= 0 || B > 65535 || nx <= 0 || ny <= 0 || nz <= 0 ||
        nx % 128 || ny % 4 || nz % 4 || Co <= 0 || Co > 16 || Co % 4 || mask < -1 || mask > 1 ||
        sample_words % 2 || sample_words / 2 < words || (uintptr_t)Y % 8 ||
        (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_pool_conv_planes_bf16: bad arguments");
    const int T = (nx / 128) * ((ny / 4 + 3) / 4) * ((nz / 4 + 1) / 2);
    const int npb = T % 32 == 0 ? 4 : 1;
    hipLaunchKernelGGL((pool_conv_labels_kernel<true, true>),
                       dim3((unsigned)((T + npb - 1) / npb), (unsigned)B), dim3(256), 0,
                       static_cast<hipStream_t>(stream), nullptr, planes, sample_words, idx, nx, ny,
                       nz, mask, mask < 0 ? 2 : 1, Co, npb, static_cast<const uint16_t *>(Wt), bias,
                       relu, Y);
    return launched("nn_pool_conv_planes_bf16");
}

int nn_pool_conv_counts_bf16(const uint8_t *counts, int B, int nx, int ny, int nz, int mask,
                             int Co, const void *Wt, const float *bias, int relu, void *Y,
                             void *stream)
{
    if (!counts || !Wt || !Y || B <= 0 || B > 65535 || nx <= 0 || ny <= 0 || nz <= 0 ||
        nx % 128 || ny % 4 || nz % 4 || Co <= 0 || Co > 16 || Co % 4 || mask < -1 || mask > 1 ||
        (uintptr_t)counts % 16 || (uintptr_t)Y % 8 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_pool_conv_counts_bf16: bad arguments");
    const int T = (nx / 128) * ((ny / 4 + 3) / 4) * ((nz / 4 + 1) / 2);
    const int npb = T < 16 ? T : 16;               // tiles per block (the weights loaded once)
    hipLaunchKernelGGL((pool_conv_counts_kernel<true>),
                       dim3((unsigned)((T + npb - 1) / npb), (unsigned)B), dim3(256), 0,
                       static_cast<hipStream_t>(stream), counts, nx, ny, nz, mask,
                       mask < 0 ? 2 : 1, Co, npb, static_cast<const uint16_t *>(Wt), bias, relu,
                       Y);
    return launched("nn_pool_conv_counts_bf16");
}

int nn_counts_conv12_bf16(const uint8_t *counts, int B, int nx, int ny, int nz, int mask,
                          const void *Wt1, const float *b1, const void *Wtm2, const float *b2,
                          void *Y, void *stream)
{
    if (!counts || !Wt1 || !Wtm2 || !Y || B <= 0 || nx <= 0 || ny <= 0 || nz <= 0 || nx % 128 ||
        ny % 32 || nz % 16 || mask < -1 || mask > 1 || (uintptr_t)counts % 16 ||
        (uintptr_t)Wtm2 % 16 || (uintptr_t)Y % 8 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_counts_conv12_bf16: bad arguments");
    const int OD2 = nz / 8;
    const int64_t cols = (int64_t)B * (nx / 128) * (ny / 32);   // 4 x 16 output columns
    // Output slices per block: all of them, halved (each chunk recomputes one first-layer
    // slice) while fewer than 2,048 blocks would fill the chip.
    int zc = OD2;
    while (zc % 2 == 0 && zc > 4 && cols * (OD2 / zc) < 2048) zc /= 2;
    const int64_t units = cols * (OD2 / zc);
    if (units >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_counts_conv12_bf16: too large");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const auto *w1 = static_cast<const uint16_t *>(Wt1);
    const auto *w2 = static_cast<const uint16_t *>(Wtm2);
    auto *y = static_cast<uint16_t *>(Y);
    if (mask < 0)
        hipLaunchKernelGGL(counts_conv12_kernel<2>, dim3((unsigned)units), dim3(256), 0, s, counts,
                           nx, ny, nz, mask, zc, (int)units, w1, b1, w2, b2, y);
    else
        hipLaunchKernelGGL(counts_conv12_kernel<1>, dim3((unsigned)units), dim3(256), 0, s, counts,
                           nx, ny, nz, mask, zc, (int)units, w1, b1, w2, b2, y);
    return launched("nn_counts_conv12_bf16");
}

int nn_conv34_bf16(int B, const void *X, const void *Wtm3, const float *b3, const void *Wtm4,
                   const float *b4, float *Y, void *stream)
{
    if (B <= 0 || !X || !Wtm3 || !Wtm4 || !Y || (uintptr_t)X % 16 || (uintptr_t)Wtm3 % 16 ||
        (uintptr_t)Wtm4 % 16)
        return tdb_set_error(DB_EINVAL, "nn_conv34_bf16: bad arguments");
    hipLaunchKernelGGL(conv34_kernel, dim3((unsigned)B), dim3(512), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint16_t *>(X),
                       static_cast<const uint16_t *>(Wtm3), b3, static_cast<const uint16_t *>(Wtm4),
                       b4, Y);
    return launched("nn_conv34_bf16");
}

int nn_conv3d_weights_tapmajor(const void *Wt, int Co, int Ci, void *out, void *stream)
{
    if (!Wt || !out || Co <= 0 || Ci <= 0 || (int64_t)Co * Ci * 28 >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_conv3d_weights_tapmajor: bad arguments");
    const int64_t n = (int64_t)Co * 28 * Ci;
    hipLaunchKernelGGL(conv_w_tapmajor_kernel, dim3(grid1(n, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), Co, Ci, static_cast<const uint16_t *>(Wt),
                       static_cast<uint16_t *>(out));
    return launched("nn_conv3d_weights_tapmajor");
}

int nn_conv3d_s2_fwd_bf16(int B, int Ci, int Co, int D, int H, int W, const void *X,
                          const void *Wtm, const float *bias, int relu, int out_f32, void *Y,
                          void *stream)
{
    // Output box per block for each supported (Ci, Co).
    int TD = 0, TH = 0, TW = 0;
    if (Ci == 8 && Co == 16) TD = 2, TH = 4, TW = 16;
    else if (Ci == 16 && Co == 32) TD = 4, TH = 4, TW = 8;
    else if (Ci == 32 && Co == 64) TD = 4, TH = 4, TW = 4;
    if (!TD || !X || !Wtm || !Y || B <= 0 || B > 65535 || D <= 0 || H <= 0 || W <= 0 ||
        D % (2 * TD) || H % (2 * TH) || W % (2 * TW) || (uintptr_t)X % 16 || (uintptr_t)Wtm % 16 ||
        (uintptr_t)Y % 8 || (int64_t)D * H * W * Ci >= ((int64_t)1 << 31))
        return tdb_set_error(DB_EINVAL, "nn_conv3d_s2_fwd_bf16: bad arguments");
    const int th = H / 2 / TH, tw = W / 2 / TW;
    const int64_t T = (int64_t)B * (D / 2 / TD) * th * tw;   // tiles over all samples
    if (T >= ((int64_t)1 << 31)) return tdb_set_error(DB_EINVAL, "nn_conv3d_s2_fwd_bf16: too large");
    // Tiles per block (the next one prefetched), while at least 2,048 blocks remain.
    const int npb = (int)std::max<int64_t>(1, std::min<int64_t>(4, T / 2048));
    const dim3 grid((unsigned)((T + npb - 1) / npb));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const auto *x = static_cast<const uint16_t *>(X);
    const auto *w = static_cast<const uint16_t *>(Wtm);
#define TDB_CONV_BF16(CI_, CO_, TD_, TH_, TW_)                                                      \
    do {                                                                                           \
        if (out_f32)                                                                               \
            hipLaunchKernelGGL((conv_bf16_kernel<CI_, CO_, TD_, TH_, TW_, true>), grid, dim3(256), \
                               0, s, D, H, W, th, tw, (int)T, npb, x, w, bias, relu, Y);         \
        else                                                                                       \
            hipLaunchKernelGGL((conv_bf16_kernel<CI_, CO_, TD_, TH_, TW_, false>), grid,           \
                               dim3(256), 0, s, D, H, W, th, tw, (int)T, npb, x, w, bias, relu, Y); \
    } while (0)
    if (Ci == 8) TDB_CONV_BF16(8, 16, 2, 4, 16);
    else if (Ci == 16) TDB_CONV_BF16(16, 32, 4, 4, 8);
    else TDB_CONV_BF16(32, 64, 4, 4, 4);
#undef TDB_CONV_BF16
    return launched("nn_conv3d_s2_fwd_bf16");
}

int nn_conv3d_s2_fwd(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *X,
                     const void *Wt, int wdtype, const void *bias, int relu, void *Y, void *stream)
{
    const int pair = dtype_pair(dtype, wdtype);
    if (pair < 0 || !conv_dims_ok(B, Ci, Co, D, H, W) || !X || !Wt || !Y)
        return tdb_set_error(DB_EINVAL, "nn_conv3d_s2_fwd: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (pair <= 1 && Ci % 4 == 0 && W % 4 == 0 && (uintptr_t)X % 16 == 0 && Co <= 64 &&
        B <= 65535 && (int64_t)D * H * W * 4 < ((int64_t)1 << 31)) {
        const int e = conv_fwd_mfma(pair == 0, B, Ci, Co, D, H, W, X, Wt, bias, relu, Y, s);
        if (e <= 0) return e;                     // launched (or failed); > 0: shape not covered
    }
    const int64_t osp = (int64_t)(D / 2) * (H / 2) * (W / 2);
    // 16 output channels per thread for the small late layers (Co >= 16, at most 16^3
    // input voxels): every input tap loaded then feeds twice the multiply-adds. The
    // large early layers keep 8, which leaves room for more waves per SIMD.
    const bool wide = Co >= 16 && (int64_t)D * H * W <= 4096;
    const int cb = wide ? 16 : kCB;
    // Two adjacent outputs per thread on the first layer (few input channels, the
    // largest grid, even output rows): the shared input taps are loaded once.
    const int vx = (!wide && Ci <= 2 && (W / 2) % 2 == 0) ? 2 : 1;
    const dim3 grid((unsigned)((B * osp / vx + 255) / 256), (Co + cb - 1) / cb);
#define TDB_CONV_FWD(T_, WT_, CB_)                                                                 \
    do {                                                                                           \
        if (vx == 2)                                                                               \
            hipLaunchKernelGGL((conv_fwd_kernel<T_, WT_, CB_, 2>), grid, dim3(256), 0, s, B, Ci, Co, \
                               D, H, W, (const T_ *)X, (const WT_ *)Wt, (const T_ *)bias, relu,    \
                               (T_ *)Y);                                                           \
        else                                                                                       \
            hipLaunchKernelGGL((conv_fwd_kernel<T_, WT_, CB_, 1>), grid, dim3(256), 0, s, B, Ci, Co, \
                               D, H, W, (const T_ *)X, (const WT_ *)Wt, (const T_ *)bias, relu,    \
                               (T_ *)Y);                                                           \
    } while (0)
    if (pair == 0) {
        if (wide) TDB_CONV_FWD(float, uint16_t, 16); else TDB_CONV_FWD(float, uint16_t, kCB);
    } else if (pair == 1) {
        if (wide) TDB_CONV_FWD(float, float, 16); else TDB_CONV_FWD(float, float, kCB);
    } else {
        if (wide) TDB_CONV_FWD(double, double, 16); else TDB_CONV_FWD(double, double, kCB);
    }
#undef TDB_CONV_FWD
    return launched("nn_conv3d_s2_fwd");
}

int nn_conv3d_s2_bwd_data(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *dY,
                          const void *Wt, int wdtype, const void *bias, int relu, void *dX,
                          void *stream)
{
    const int pair = dtype_pair(dtype, wdtype);
    if (pair < 0 || !conv_dims_ok(B, Ci, Co, D, H, W) || !dY || !Wt || !dX)
        return tdb_set_error(DB_EINVAL, "nn_conv3d_s2_bwd_data: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t isp = (int64_t)D * H * W;
    const dim3 grid((unsigned)((B * isp + 255) / 256), (Ci + kCB - 1) / kCB);
    if (pair == 0)
        hipLaunchKernelGGL((conv_bwd_data_kernel<float, uint16_t>), grid, dim3(256), 0, s, B, Ci, Co,
                           D, H, W, (const float *)dY, (const uint16_t *)Wt, (const float *)bias,
                           relu, (float *)dX);
    else if (pair == 1)
        hipLaunchKernelGGL((conv_bwd_data_kernel<float, float>), grid, dim3(256), 0, s, B, Ci, Co, D,
                           H, W, (const float *)dY, (const float *)Wt, (const float *)bias, relu,
                           (float *)dX);
    else
        hipLaunchKernelGGL((conv_bwd_data_kernel<double, double>), grid, dim3(256), 0, s, B, Ci, Co,
                           D, H, W, (const double *)dY, (const double *)Wt, (const double *)bias,
                           relu, (double *)dX);
    return launched("nn_conv3d_s2_bwd_data");
}

size_t nn_conv3d_s2_bwd_weight_ws_bytes(int dtype, int B, int Ci, int Co, int D, int H, int W)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || !conv_dims_ok(B, Ci, Co, D, H, W)) return 0;
    const int64_t P = (int64_t)B * (D / 2) * (H / 2) * (W / 2);
    const int64_t chunks = (P + kWgChunk - 1) / kWgChunk;
    return (size_t)chunks * Co * Ci * 28 * (dtype == NN_F32 ? 4 : 8);
}

int nn_conv3d_s2_bwd_weight(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *X,
                            const void *dY, void *dWt, void *dbias, void *ws, size_t ws_bytes,
                            void *stream)
{
    const size_t need = nn_conv3d_s2_bwd_weight_ws_bytes(dtype, B, Ci, Co, D, H, W);
    if (need == 0 || !X || !dY || !dWt || !ws)
        return tdb_set_error(DB_EINVAL, "nn_conv3d_s2_bwd_weight: bad arguments");
    if (ws_bytes < need)
        return tdb_set_error(DB_ENOSPC, "nn_conv3d_s2_bwd_weight: workspace %zu < %zu", ws_bytes,
                             need);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t P = (int64_t)B * (D / 2) * (H / 2) * (W / 2);
    const int chunks = (int)((P + kWgChunk - 1) / kWgChunk);
    constexpr int kWgCB = 4;   // output channels per thread (float)
    const dim3 g1(chunks, Ci, Co);
    const dim3 g1f(chunks, Ci, (Co + kWgCB - 1) / kWgCB);
    const unsigned g2 = (unsigned)((Co * Ci * 28 + 255) / 256);
    if (dtype == NN_F32) {
        hipLaunchKernelGGL((conv_bwd_weight_partial<float, kWgCB>), g1f, dim3(256), 0, s, B, Ci, Co,
                           D, H, W, (const float *)X, (const float *)dY, (float *)ws);
        hipLaunchKernelGGL(conv_bwd_weight_final<float>, dim3(g2), dim3(256), 0, s, chunks, Ci, Co,
                           (const float *)ws, (float *)dWt, (float *)dbias);
    } else {
        hipLaunchKernelGGL((conv_bwd_weight_partial<double, 1>), g1, dim3(256), 0, s, B, Ci, Co, D,
                           H, W, (const double *)X, (const double *)dY, (double *)ws);
        hipLaunchKernelGGL(conv_bwd_weight_final<double>, dim3(g2), dim3(256), 0, s, chunks, Ci,
                           Co, (const double *)ws, (double *)dWt, (double *)dbias);
    }
    return launched("nn_conv3d_s2_bwd_weight");
}

int nn_linear_fwd_split(int B, int In, int Out, const float *X, const void *Wt,
                        const float *bias, int relu, float *Y, int splits, float *ws,
                        size_t ws_bytes, void *stream)
{
    if (B <= 0 || In <= 0 || Out <= 0 || B > 65535 || !X || !Wt || !Y || !ws || splits < 1 ||
        splits > 64 || In % 4 || (uintptr_t)X % 16 || (uintptr_t)Wt % 8)
        return tdb_set_error(DB_EINVAL, "nn_linear_fwd_split: bad arguments");
    // K per slice: a multiple of the staging step; trailing slices may be empty (zero sums).
    const int kc = (In + splits * kMK - 1) / (splits * kMK) * kMK;
    if (ws_bytes < (size_t)splits * B * Out * sizeof(float))
        return tdb_set_error(DB_ENOSPC, "nn_linear_fwd_split: workspace %zu bytes < %zu needed",
                             ws_bytes, (size_t)splits * B * Out * sizeof(float));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 mgrid((Out + kMM - 1) / kMM, (B + kMM - 1) / kMM, splits);
    hipLaunchKernelGGL((linear_mfma_kernel<uint16_t, false, true>), mgrid, dim3(512), 0, s, B,
                       Out, In, X, (const uint16_t *)Wt, nullptr, 0, ws, kc);
    const int64_t MN = (int64_t)B * Out;
    hipLaunchKernelGGL(linear_split_final_kernel, dim3((unsigned)std::min<int64_t>((MN + 255) / 256, 4096)),
                       dim3(256), 0, s, MN, Out, splits, (const float *)ws, bias, relu, Y);
    return launched("nn_linear_fwd_split");
}

int nn_linear_fwd(int dtype, int B, int In, int Out, const void *X, const void *Wt, int wdtype,
                  const void *bias, int relu, void *Y, void *stream)
{
    const int pair = dtype_pair(dtype, wdtype);
    if (pair < 0 || B <= 0 || In <= 0 || Out <= 0 || B > 65535 || !X || !Wt || !Y)
        return tdb_set_error(DB_EINVAL, "nn_linear_fwd: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid((Out + kLN - 1) / kLN, (B + kLM - 1) / kLM);
    const dim3 mgrid((Out + kMM - 1) / kMM, (B + kMM - 1) / kMM);
    // The matrix-core path loads four k at a time: rows and bases must be aligned to that.
    const size_t wal = pair == 0 ? 8 : 16;
    const bool vec = In % 4 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)Wt % wal == 0;
    if (pair == 0 && vec)
        hipLaunchKernelGGL((linear_mfma_kernel<uint16_t, false>), mgrid, dim3(512), 0, s, B, Out, In,
                           (const float *)X, (const uint16_t *)Wt, (const float *)bias, relu,
                           (float *)Y);
    else if (pair == 1 && vec)
        hipLaunchKernelGGL((linear_mfma_kernel<float, false>), mgrid, dim3(512), 0, s, B, Out, In,
                           (const float *)X, (const float *)Wt, (const float *)bias, relu,
                           (float *)Y);
    else if (pair == 0)
        hipLaunchKernelGGL((linear_gemm_kernel<float, uint16_t, false>), grid, dim3(256), 0, s, B,
                           Out, In, (const float *)X, (const uint16_t *)Wt, (const float *)bias,
                           relu, (float *)Y);
    else if (pair == 1)
        hipLaunchKernelGGL((linear_gemm_kernel<float, float, false>), grid, dim3(256), 0, s, B, Out,
                           In, (const float *)X, (const float *)Wt, (const float *)bias, relu,
                           (float *)Y);
    else
        hipLaunchKernelGGL((linear_gemm_kernel<double, double, false>), grid, dim3(256), 0, s, B,
                           Out, In, (const double *)X, (const double *)Wt, (const double *)bias,
                           relu, (double *)Y);
    return launched("nn_linear_fwd");
}

int nn_linear_bwd_data(int dtype, int B, int In, int Out, const void *dY, const void *Wt,
                       int wdtype, void *dX, void *stream)
{
    const int pair = dtype_pair(dtype, wdtype);
    if (pair < 0 || B <= 0 || In <= 0 || Out <= 0 || B > 65535 || !dY || !Wt || !dX)
        return tdb_set_error(DB_EINVAL, "nn_linear_bwd_data: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid((In + kLN - 1) / kLN, (B + kLM - 1) / kLM);
    const dim3 mgrid((In + kMM - 1) / kMM, (B + kMM - 1) / kMM);
    // Matrix-core path: dY rows (K = Out) and W rows (N = In) in groups of four.
    const size_t wal = pair == 0 ? 8 : 16;
    const bool vec = In % 4 == 0 && Out % 4 == 0 && (uintptr_t)dY % 16 == 0 &&
                     (uintptr_t)Wt % wal == 0;
    if (pair == 0 && vec)
        hipLaunchKernelGGL((linear_mfma_kernel<uint16_t, true>), mgrid, dim3(512), 0, s, B, In, Out,
                           (const float *)dY, (const uint16_t *)Wt, (const float *)nullptr, 0,
                           (float *)dX);
    else if (pair == 1 && vec)
        hipLaunchKernelGGL((linear_mfma_kernel<float, true>), mgrid, dim3(512), 0, s, B, In, Out,
                           (const float *)dY, (const float *)Wt, (const float *)nullptr, 0,
                           (float *)dX);
    else if (pair == 0)
        hipLaunchKernelGGL((linear_gemm_kernel<float, uint16_t, true>), grid, dim3(256), 0, s, B, In,
                           Out, (const float *)dY, (const uint16_t *)Wt, (const float *)nullptr, 0,
                           (float *)dX);
    else if (pair == 1)
        hipLaunchKernelGGL((linear_gemm_kernel<float, float, true>), grid, dim3(256), 0, s, B, In,
                           Out, (const float *)dY, (const float *)Wt, (const float *)nullptr, 0,
                           (float *)dX);
    else
        hipLaunchKernelGGL((linear_gemm_kernel<double, double, true>), grid, dim3(256), 0, s, B, In,
                           Out, (const double *)dY, (const double *)Wt, (const double *)nullptr, 0,
                           (double *)dX);
    return launched("nn_linear_bwd_data");
}

int nn_linear_bwd_weight(int dtype, int B, int In, int Out, const void *X, const void *dY,
                         void *dWt, void *dbias, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || In <= 0 || Out <= 0 || Out > 65535 ||
        !X || !dY || !dWt)
        return tdb_set_error(DB_EINVAL, "nn_linear_bwd_weight: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid((In + 255) / 256, Out);
    if (dtype == NN_F32)
        hipLaunchKernelGGL(linear_bwd_weight_kernel<float>, grid, dim3(256), 0, s, B, In, Out,
                           (const float *)X, (const float *)dY, (float *)dWt, (float *)dbias);
    else
        hipLaunchKernelGGL(linear_bwd_weight_kernel<double>, grid, dim3(256), 0, s, B, In, Out,
                           (const double *)X, (const double *)dY, (double *)dWt, (double *)dbias);
    return launched("nn_linear_bwd_weight");
}

size_t nn_channel_sum_ws_bytes(int dtype, int B, int C, int64_t S)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || B <= 0 || C <= 0 || S <= 0) return 0;
    const int64_t chunks = ((int64_t)B * S + kCsChunk - 1) / kCsChunk;
    return (size_t)chunks * C * (dtype == NN_F32 ? 4 : 8);
}

int nn_channel_sum(int dtype, int B, int C, int64_t S, const void *X, void *out, void *ws,
                   size_t ws_bytes, void *stream)
{
    const size_t need = nn_channel_sum_ws_bytes(dtype, B, C, S);
    if (need == 0 || !X || !out || !ws || C > 65535)
        return tdb_set_error(DB_EINVAL, "nn_channel_sum: bad arguments");
    if (ws_bytes < need) return tdb_set_error(DB_ENOSPC, "nn_channel_sum: workspace too small");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int chunks = (int)(((int64_t)B * S + kCsChunk - 1) / kCsChunk);
    if (dtype == NN_F32) {
        hipLaunchKernelGGL(channel_sum_partial<float>, dim3(chunks, C), dim3(256), 0, s, B, C, S,
                           (const float *)X, (float *)ws);
        hipLaunchKernelGGL(channel_sum_final<float>, dim3((C + 63) / 64), dim3(64), 0, s, C, chunks,
                           (const float *)ws, (float *)out);
    } else {
        hipLaunchKernelGGL(channel_sum_partial<double>, dim3(chunks, C), dim3(256), 0, s, B, C, S,
                           (const double *)X, (double *)ws);
        hipLaunchKernelGGL(channel_sum_final<double>, dim3((C + 63) / 64), dim3(64), 0, s, C,
                           chunks, (const double *)ws, (double *)out);
    }
    return launched("nn_channel_sum");
}

int nn_relu_bwd(int dtype, int64_t n, const void *Y, const void *dY, void *dX, void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || n <= 0 || !Y || !dY || !dX)
        return tdb_set_error(DB_EINVAL, "nn_relu_bwd: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == NN_F32)
        hipLaunchKernelGGL(relu_bwd_kernel<float>, dim3(grid1(n)), dim3(256), 0, s, n,
                           (const float *)Y, (const float *)dY, (float *)dX);
    else
        hipLaunchKernelGGL(relu_bwd_kernel<double>, dim3(grid1(n)), dim3(256), 0, s, n,
                           (const double *)Y, (const double *)dY, (double *)dX);
    return launched("nn_relu_bwd");
}

size_t nn_mse_ws_bytes(int dtype, int64_t n)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || n <= 0) return 0;
    return (size_t)kMseBlocks * (dtype == NN_F32 ? 4 : 8);
}

int nn_mse_fwd(int dtype, int64_t n, const void *A, const void *B, void *loss, void *ws,
               size_t ws_bytes, void *stream)
{
    const size_t need = nn_mse_ws_bytes(dtype, n);
    if (need == 0 || !A || !B || !loss || !ws)
        return tdb_set_error(DB_EINVAL, "nn_mse_fwd: bad arguments");
    if (ws_bytes < need) return tdb_set_error(DB_ENOSPC, "nn_mse_fwd: workspace too small");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == NN_F32) {
        hipLaunchKernelGGL(mse_partial_kernel<float>, dim3(kMseBlocks), dim3(256), 0, s, n,
                           (const float *)A, (const float *)B, (float *)ws);
        hipLaunchKernelGGL(mse_final_kernel<float>, dim3(1), dim3(64), 0, s, kMseBlocks, n,
                           (const float *)ws, (float *)loss);
    } else {
        hipLaunchKernelGGL(mse_partial_kernel<double>, dim3(kMseBlocks), dim3(256), 0, s, n,
                           (const double *)A, (const double *)B, (double *)ws);
        hipLaunchKernelGGL(mse_final_kernel<double>, dim3(1), dim3(64), 0, s, kMseBlocks, n,
                           (const double *)ws, (double *)loss);
    }
    return launched("nn_mse_fwd");
}

int nn_mse_bwd(int dtype, int64_t n, const void *A, const void *B, const void *g, void *dA,
               void *stream)
{
    if ((dtype != NN_F32 && dtype != NN_F64) || n <= 0 || !A || !B || !g || !dA)
        return tdb_set_error(DB_EINVAL, "nn_mse_bwd: bad arguments");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == NN_F32)
        hipLaunchKernelGGL(mse_bwd_kernel<float>, dim3(grid1(n)), dim3(256), 0, s, n,
                           (const float *)A, (const float *)B, (const float *)g, (float *)dA);
    else
        hipLaunchKernelGGL(mse_bwd_kernel<double>, dim3(grid1(n)), dim3(256), 0, s, n,
                           (const double *)A, (const double *)B, (const double *)g, (double *)dA);
    return launched("nn_mse_bwd");
}

int nn_adam_step(int64_t n, float *w, float *m, float *v, const float *g, uint16_t *w_bf16,
                 float lr, float b1, float b2, float eps, int t, void *stream)
{
    if (n <= 0 || !w || !m || !v || !g || t < 1 || !(b1 >= 0.f && b1 < 1.f) ||
        !(b2 >= 0.f && b2 < 1.f))
        return tdb_set_error(DB_EINVAL, "nn_adam_step: bad arguments");
    const float c1 = 1.0f - powf(b1, (float)t);
    const float c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid1(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       n, w, m, v, g, w_bf16, lr, b1, b2, eps, c1, c2);
    return launched("nn_adam_step");
}

int nn_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream)
{
    if (n <= 0 || !x || !y) return tdb_set_error(DB_EINVAL, "nn_to_bf16: bad arguments");
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n, x, y);
    return launched("nn_to_bf16");
}

}  // extern "C"
