/*
 * tumornn.h — C ABI of the encoder kernels used for embedding search.
 *
 * The paper compresses each tumour with a convolutional autoencoder: strided
 * 3-D convolutions (stride 2, kernel 3) down to a small grid, a linear layer
 * to the latent, and a decoder of strided transposed convolutions mirroring
 * it (Sec. 2.4 "Implementation"; Sec. 2.3 "Autoencoders"); database and
 * query are compared by L2 distance of their latents (Sec. 2.3). The inputs
 * here are the two masks mean-pooled by 2 in every axis (the paper's
 * downsampling idea, Sec. 2.3 "Baseline for-loop search", DS64).
 *
 * Conventions:
 *  - Tensors are dense, row-major, device memory: activations [B][C][D][H][W]
 *    (W fastest), convolution weights [Co][Ci][3][3][3], linear weights
 *    [Out][In], biases [Co]. Transposed-convolution weights are [Ci][Co][3][3][3]
 *    (input channels first); see the duality notes below.
 *  - dtype codes: NN_F32, NN_F64 for activations / gradients; weights may be
 *    NN_BF16 (uint16 storage, bfloat16 bits) or NN_F32 with NN_F32
 *    activations, and must be NN_F64 with NN_F64 activations (the FP64
 *    build exists for finite-difference checks). Accumulation is in the
 *    activation type.
 *  - Return 0 on success, a negative DB_* code (tumordb.h) on bad arguments;
 *    the message is in db_last_error(). Nothing is written on error.
 *  - Calls are asynchronous on `stream` (hipStream_t as void*).
 *
 * Convolution, kernel 3, stride 2, padding 1, on even extents D, H, W:
 *   Y[b,co,o] = bias[co] + sum_{ci,k} Wt[co,ci,k] X[b,ci,2o+k-1]   (o < D/2 per axis)
 * Transposed convolution with output padding 1 (output 2x the input) is the
 * adjoint of that map: its forward is nn_conv3d_s2_bwd_data (plus a bias),
 * its input gradient is nn_conv3d_s2_fwd, and its weight gradient is
 * nn_conv3d_s2_bwd_weight with the roles of X and dY exchanged.
 */
#ifndef TUMORNN_H
#define TUMORNN_H

#include <stddef.h>
#include <stdint.h>

#include "tumordb.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { NN_F32 = 0, NN_F64 = 1, NN_BF16 = 2 };

/* 2x2x2 mean of the packed masks of database entries idx[0..B) (device
 * int32): out [B][2][nz/2][ny/2][nx/2] (dtype), channel 0 FLAIR, 1 T1Gd;
 * values are k/8 exactly. Needs even dims. */
int nn_meanpool_db(const db_t *db, const int32_t *idx, int B, void *out, int dtype, void *stream);

/* Same from query labels uint8 [B][nz][ny][nx] (bit 0 FLAIR, bit 1 T1Gd). */
int nn_meanpool_labels(const uint8_t *labels, int B, int nx, int ny, int nz, void *out, int dtype,
                       void *stream);

/* One mask only (mask 0 = FLAIR, 1 = T1Gd): out [B][1][nz/2][ny/2][nx/2], for
 * the paper's separate FLAIR and T1Gd autoencoders (Sec. 2.3). */
int nn_meanpool_db_mask(const db_t *db, const int32_t *idx, int B, int mask, void *out, int dtype,
                        void *stream);
int nn_meanpool_labels_mask(const uint8_t *labels, int B, int nx, int ny, int nz, int mask,
                            void *out, int dtype, void *stream);

/* First encoder layer read straight from query labels: Y = act(conv(P) + bias)
 * where P is the 2x2x2 mean of the masks (as nn_meanpool_labels, or
 * nn_meanpool_labels_mask for one mask) and conv the stride-2 convolution
 * below; one pass, the pooled volume never goes to memory. mask -1: P has two
 * channels (FLAIR, T1Gd), Wt is [Co][2][3][3][3]; mask 0 / 1: that mask alone,
 * Wt [Co][1][3][3][3]. Wt bfloat16 bits (uint16), bias float [Co] or NULL,
 * Y float [B][Co][nz/4][ny/4][nx/4]. Pooled values (multiples of 1/8) and
 * weights are exact in the BF16 matrix-core products, sums are FP32, so Y
 * equals the two-call result up to summation order. Needs nx % 128 == 0,
 * ny % 4 == 0, nz % 4 == 0, Co <= 16, B <= 65535, labels 16-byte aligned. */
int nn_pool_conv_labels(const uint8_t *labels, int B, int nx, int ny, int nz, int mask, int Co,
                        const void *Wt, const float *bias, int relu, float *Y, void *stream);

/* nn_pool_conv_labels from packed masks instead of label bytes: sample b's
 * masks are the LSB-first uint32 bit planes (x fastest; plane 0 FLAIR, plane 1
 * T1Gd, sample_words / 2 words each) at planes + s * sample_words with
 * s = idx[b] (device int32 [B]) or s = b when idx is NULL: the database's
 * planes (sample_words = 2 Wp, idx = entries) or the queries packed by
 * db_rerank_pack. Y equals nn_pool_conv_labels' for the labels that packed to
 * these masks, bit for bit (same pooled values, same products and order). A
 * pooled row reads 4 x 16 bits per mask instead of 4 x 16 bytes. Same shape
 * rules as nn_pool_conv_labels; sample_words even and at least
 * 2 nx ny nz / 32. */
int nn_pool_conv_planes(const uint32_t *planes, int64_t sample_words, const int32_t *idx, int B,
                        int nx, int ny, int nz, int mask, int Co, const void *Wt,
                        const float *bias, int relu, float *Y, void *stream);

/* ---- BF16 inference forward -------------------------------------------------
 * The encoder's forward for inference with bfloat16 activations stored
 * channels-last. Each layer's output is the FP32 result (BF16 x BF16 products,
 * exact in FP32, summed in FP32, plus bias, ReLU) rounded to the nearest
 * bfloat16 (ties to even); the last convolution may write float instead, in
 * the [B][Co][D][H][W] order the linear head flattens. This is a different
 * numerics contract from the float path (nn_pool_conv_labels,
 * nn_conv3d_s2_fwd): a layer's output equals the float64 result of the same
 * bfloat16 inputs and weights, rounded to bfloat16, except where the FP32 sum
 * and the exact value round to neighbouring bfloat16 values. */

/* nn_pool_conv_labels writing Y as bfloat16 channels-last [B][nz/4][ny/4][nx/4][Co]
 * (device, 8-byte aligned); also needs Co % 4 == 0. Same arguments otherwise. */
int nn_pool_conv_labels_bf16(const uint8_t *labels, int B, int nx, int ny, int nz, int mask,
                             int Co, const void *Wt, const float *bias, int relu, void *Y,
                             void *stream);
/* nn_pool_conv_planes with the output of nn_pool_conv_labels_bf16 (bit for bit the same
 * for the labels that packed to these masks). */
int nn_pool_conv_planes_bf16(const uint32_t *planes, int64_t sample_words, const int32_t *idx,
                             int B, int nx, int ny, int nz, int mask, int Co, const void *Wt,
                             const float *bias, int relu, void *Y, void *stream);
/* nn_pool_conv_labels_bf16 from the pooled counts that db_rerank_pack_pool writes:
 * counts uint8 [B][nz/2][ny/2][nx/2] (device, 16-byte aligned), per 2x2x2 block of voxels
 * the FLAIR count (0..8) in bits 0..3 and the T1Gd count in bits 4..7. The pooled means
 * are counts / 8 (Sec. 2.3, "Autoencoders": the input halved by mean pooling), so Y equals
 * nn_pool_conv_labels_bf16's for the labels the counts came from, bit for bit; the labels
 * are not read again. Same arguments and rules otherwise. */
int nn_pool_conv_counts_bf16(const uint8_t *counts, int B, int nx, int ny, int nz, int mask,
                             int Co, const void *Wt, const float *bias, int relu, void *Y,
                             void *stream);
/* The encoder's first two layers in one pass (Sec. 2.3, "Autoencoders": the convolutions of
 * the halved input): nn_pool_conv_counts_bf16 with Co = 8 and ReLU, then
 * nn_conv3d_s2_fwd_bf16 with (Ci, Co) = (8, 16) and ReLU, bit for bit, without the first
 * layer's activations leaving the chip. counts uint8 [B][nz/2][ny/2][nx/2] as for
 * nn_pool_conv_counts_bf16 (16-byte aligned); Wt1 bfloat16 [8][Ci][27] (Ci = 2, or 1 with
 * mask = 0 / 1 as there); b1 float [8] or NULL; Wtm2 the tap-major bfloat16 second-layer
 * weights [16][28][8] of nn_conv3d_weights_tapmajor (16-byte aligned); b2 float [16] or NULL;
 * Y bfloat16 channels-last [B][nz/8][ny/8][nx/8][16] (8-byte aligned). nx % 128 == 0,
 * ny % 32 == 0, nz % 16 == 0 (the grids of the two kernels), nx * ny * nz < 2^31;
 * DB_EINVAL otherwise. All device
 * pointers, owned by the caller; enqueued on `stream`. */
int nn_counts_conv12_bf16(const uint8_t *counts, int B, int nx, int ny, int nz, int mask,
                          const void *Wt1, const float *b1, const void *Wtm2, const float *b2,
                          void *Y, void *stream);
/* The encoder's third and fourth layers in one pass (Sec. 2.3, "Autoencoders"), one block per
 * sample: nn_conv3d_s2_fwd_bf16 with (Ci, Co) = (16, 32), ReLU, bfloat16 output, then with
 * (32, 64), ReLU, float output, bit for bit, the third layer's output kept on chip.
 * X bfloat16 channels-last [B][16][16][16][16] (16-byte aligned); Wtm3 / Wtm4 the tap-major
 * weights [32][28][16] / [64][28][32] of nn_conv3d_weights_tapmajor (16-byte aligned); b3 [32]
 * and b4 [64] float or NULL; Y float [B][64][4][4][4]. Device pointers, caller-owned;
 * enqueued on `stream`. DB_EINVAL for B <= 0, a NULL or misaligned pointer. */
int nn_conv34_bf16(int B, const void *X, const void *Wtm3, const float *b3, const void *Wtm4,
                   const float *b4, float *Y, void *stream);
/* Tap-major copy of bfloat16 convolution weights for nn_conv3d_s2_fwd_bf16:
 * out[co][t][ci] = Wt[co][ci][t] for the 27 taps t (kd, kh, kw order) and 0 for
 * t = 27; out holds Co * 28 * Ci bfloat16 values (device). */
int nn_conv3d_weights_tapmajor(const void *Wt, int Co, int Ci, void *out, void *stream);
/* Y = act(conv(X) + bias), stride 2, padding 1, kernel 3, on the BF16 matrix
 * cores. X bfloat16 channels-last [B][D][H][W][Ci] (16-byte aligned); Wtm the
 * tap-major weights of nn_conv3d_weights_tapmajor (16-byte aligned); bias float
 * [Co] or NULL; Y bfloat16 channels-last [B][D/2][H/2][W/2][Co], or with
 * out_f32 float [B][Co][D/2][H/2][W/2] (8-byte aligned). (Ci, Co) one of
 * (8, 16), (16, 32), (32, 64), whose output boxes per block are 2 x 4 x 16,
 * 4 x 4 x 8 and 4 x 4 x 4: D/2, H/2, W/2 must be multiples of them;
 * B <= 65535. DB_EINVAL otherwise. */
int nn_conv3d_s2_fwd_bf16(int B, int Ci, int Co, int D, int H, int W, const void *X,
                          const void *Wtm, const float *bias, int relu, int out_f32, void *Y,
                          void *stream);

/* Y = act(conv(X)) with X [B][Ci][D][H][W], Y [B][Co][D/2][H/2][W/2];
 * bias [Co] or NULL; relu != 0 applies max(0, .). */
int nn_conv3d_s2_fwd(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *X,
                     const void *Wt, int wdtype, const void *bias, int relu, void *Y,
                     void *stream);

/* dX = conv^T(dY) (the adjoint map; also the transposed-convolution forward):
 * dY [B][Co][D/2][H/2][W/2] -> dX [B][Ci][D][H][W]; bias [Ci] or NULL is added
 * and relu != 0 applied (used only as a transposed-convolution forward). */
int nn_conv3d_s2_bwd_data(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *dY,
                          const void *Wt, int wdtype, const void *bias, int relu, void *dX,
                          void *stream);

/* dWt[co,ci,k] = sum_{b,o} dY[b,co,o] X[b,ci,2o+k-1] and dbias[co] = sum dY
 * (dbias may be NULL). Deterministic two-stage reduction through ws. */
size_t nn_conv3d_s2_bwd_weight_ws_bytes(int dtype, int B, int Ci, int Co, int D, int H, int W);
int nn_conv3d_s2_bwd_weight(int dtype, int B, int Ci, int Co, int D, int H, int W, const void *X,
                            const void *dY, void *dWt, void *dbias, void *ws, size_t ws_bytes,
                            void *stream);

/* Y[b,j] = act(bias[j] + sum_i Wt[j,i] X[b,i]); X [B][In], Wt [Out][In]. */
int nn_linear_fwd(int dtype, int B, int In, int Out, const void *X, const void *Wt, int wdtype,
                  const void *bias, int relu, void *Y, void *stream);
/* nn_linear_fwd for float X and bfloat16 Wt on the FP32 matrix cores with K split into
 * `splits` slices, so that a small batch still fills the GPU: slice z sums k in
 * [z kc, (z + 1) kc) (kc = In / splits rounded up to a multiple of 64) into ws
 * (float [splits][B][Out], device, ws_bytes >= 4 splits B Out), then a second kernel adds
 * the slices in order z = 0, 1, ..., adds the bias and applies the ReLU. Deterministic; with
 * splits = 1 equal to nn_linear_fwd bit for bit, otherwise within the same FP32 sum bound.
 * Needs In % 4 == 0, X 16-byte and Wt 8-byte aligned, 1 <= splits <= 64, B <= 65535;
 * DB_EINVAL / DB_ENOSPC otherwise. */
int nn_linear_fwd_split(int B, int In, int Out, const float *X, const void *Wt,
                        const float *bias, int relu, float *Y, int splits, float *ws,
                        size_t ws_bytes, void *stream);
/* dX[b,i] = sum_j Wt[j,i] dY[b,j]. */
int nn_linear_bwd_data(int dtype, int B, int In, int Out, const void *dY, const void *Wt,
                       int wdtype, void *dX, void *stream);
/* dWt[j,i] = sum_b dY[b,j] X[b,i]; dbias[j] = sum_b dY[b,j] (or NULL). */
int nn_linear_bwd_weight(int dtype, int B, int In, int Out, const void *X, const void *dY,
                         void *dWt, void *dbias, void *stream);

/* out[c] = sum_{b,s} X[b][c][s] for X [B][C][S] (a bias gradient); two fixed-order
 * stages through ws of nn_channel_sum_ws_bytes bytes. */
size_t nn_channel_sum_ws_bytes(int dtype, int B, int C, int64_t S);
int nn_channel_sum(int dtype, int B, int C, int64_t S, const void *X, void *out, void *ws,
                   size_t ws_bytes, void *stream);

/* dX = dY where Y > 0 else 0 (n elements). */
int nn_relu_bwd(int dtype, int64_t n, const void *Y, const void *dY, void *dX, void *stream);

/* loss[0] = mean((A - B)^2) over n elements (deterministic; ws of
 * nn_mse_ws_bytes(n) bytes). */
size_t nn_mse_ws_bytes(int dtype, int64_t n);
int nn_mse_fwd(int dtype, int64_t n, const void *A, const void *B, void *loss, void *ws,
               size_t ws_bytes, void *stream);
/* dA = g[0] * 2 (A - B) / n, with g a device scalar (the upstream gradient). */
int nn_mse_bwd(int dtype, int64_t n, const void *A, const void *B, const void *g, void *dA,
               void *stream);

/* Adam (Kingma & Ba) on FP32 master weights, then the BF16 copy (round to
 * nearest even): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); w_bf16 may be NULL. */
int nn_adam_step(int64_t n, float *w, float *m, float *v, const float *g, uint16_t *w_bf16,
                 float lr, float b1, float b2, float eps, int t, void *stream);

/* The Bi-half hash layer of the paper's hashing autoencoder (Sec. 2.3): for
 * U [B][D] (NN_F32 or NN_F64), out[i][d] = +1 if row i is among the first
 * floor(B/2) rows of column d ordered by (value desc, row asc), else -1.
 * Backward (a surrogate, the layer is piecewise constant): the incoming
 * gradient passes straight through, plus a pull of U towards its code:
 * dU = G + gamma * ((U - Bc) / (B * D)), each operation rounded in the dtype
 * in that order. B <= 4096. */
int nn_bihalf_fwd(int dtype, int B, int D, const void *U, void *out, void *stream);
int nn_bihalf_bwd(int dtype, int B, int D, double gamma, const void *U, const void *Bc,
                  const void *G, void *dU, void *stream);

/* Variational head of the paper's VAE (Sec. 2.3 "Autoencoders", Sec. 2.4: two
 * linear layers give the latent mean and log-variance). ML [B][2L]: row b is
 * mu_b (L values) then logvar_b (L values), as one linear layer of 2L outputs
 * writes them. Forward: z [B][L] = mu + exp(logvar / 2) * eps (eps [B][L], a
 * standard normal sample passed in), kl[0] = (1/B) sum -1/2 (1 + logvar - mu^2
 * - exp(logvar)) (deterministic: fixed-order partial sums in ws of
 * nn_vae_ws_bytes bytes). Backward of recon(z) + beta * kl, given dz:
 *   d mu = dz + beta * mu / B,
 *   d logvar = dz * eps * exp(logvar / 2) / 2 + beta * (exp(logvar) - 1) / (2B),
 * written to dML [B][2L]. dtype NN_F32 or NN_F64. */
size_t nn_vae_ws_bytes(int dtype, int B, int L);
int nn_vae_head_fwd(int dtype, int B, int L, const void *ML, const void *eps, void *z, void *kl,
                    void *ws, size_t ws_bytes, void *stream);
int nn_vae_head_bwd(int dtype, int B, int L, double beta, const void *ML, const void *eps,
                    const void *dz, void *dML, void *stream);

/* FP32 -> BF16 bits, round to nearest even (NaN stays NaN). */
int nn_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TUMORNN_H */
