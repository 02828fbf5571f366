"""CPU oracle of the embedding path: mean-pooling, autoencoder forward, latent distances.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Follows the paper's compression strategies (Sec. 2.3): downsampling of the
volumes (DS64) and an autoencoder made of strided 3-D convolutions (stride 2,
kernel 3), a linear layer to the latent, and a mirrored decoder of strided
transposed convolutions (Sec. 2.4 "Implementation"); latents are compared by
L2 distance, lowest wins (Sec. 2.3). Written with plain torch CPU operations
in float64 (conv3d / conv_transpose3d / linear are library primitives used
as single steps) and numpy.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def meanpool(labels: np.ndarray) -> np.ndarray:
    """uint8 labels [B][nz][ny][nx] -> float64 [B][2][nz/2][ny/2][nx/2]: mean of each 2x2x2 block
    of the FLAIR (bit 0) and T1Gd (bit 1) masks."""
    lab = np.asarray(labels)
    if lab.ndim == 3:
        lab = lab[None]
    B, nz, ny, nx = lab.shape
    out = np.empty((B, 2, nz // 2, ny // 2, nx // 2), dtype=np.float64)
    for m in range(2):
        bit = ((lab >> m) & 1).astype(np.float64)
        out[:, m] = bit.reshape(B, nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4, 6))
    return out


def conv(x, w, b, relu):
    """Stride-2, padding-1 convolution with a 3x3x3 kernel, then optional ReLU (float64, CPU)."""
    y = F.conv3d(x, w, b, stride=2, padding=1)
    return torch.relu(y) if relu else y


def conv_t(x, w, b, relu):
    """Stride-2 transposed convolution, padding 1, output padding 1 (output twice the input)."""
    y = F.conv_transpose3d(x, w, b, stride=2, padding=1, output_padding=1)
    return torch.relu(y) if relu else y


def encode(params: dict, x: torch.Tensor) -> torch.Tensor:
    """Latent of x [B][2][g][g][g]: four ReLU convolutions, flatten, linear (no activation)."""
    h = x
    for i in range(4):
        h = conv(h, params[f"enc{i}.w"], params[f"enc{i}.b"], True)
    return F.linear(h.reshape(h.shape[0], -1), params["enc_fc.w"], params["enc_fc.b"])


def round_bf16(t: torch.Tensor) -> torch.Tensor:
    """The bfloat16 storage of a layer output: each value rounded to float32 (nearest, ties
    to even), then to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.asarray(t.detach().cpu().numpy(), dtype=np.float64).astype(np.float32)
    return torch.from_numpy(bf16_decode(bf16_encode(a)).reshape(a.shape))


def encode_bf16_activations(params: dict, x: torch.Tensor) -> torch.Tensor:
    """encode with bfloat16 activation storage between the convolutions: the output of each
    of the first three convolutions (after bias and ReLU) is rounded by round_bf16 before the
    next layer reads it; the last convolution and the linear layer are as in encode."""
    h = x
    for i in range(4):
        h = conv(h, params[f"enc{i}.w"], params[f"enc{i}.b"], True)
        if i < 3:
            h = round_bf16(h)
    return F.linear(h.reshape(h.shape[0], -1), params["enc_fc.w"], params["enc_fc.b"])


def decode(params: dict, z: torch.Tensor, channels: int, s: int) -> torch.Tensor:
    """Linear (ReLU), reshape to [channels][s][s][s], four transposed convolutions (ReLU but the last)."""
    h = torch.relu(F.linear(z, params["dec_fc.w"], params["dec_fc.b"]))
    h = h.reshape(h.shape[0], channels, s, s, s)
    for i in reversed(range(4)):
        h = conv_t(h, params[f"dec{i}.w"], params[f"dec{i}.b"], i != 0)
    return h


def mse(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return ((a - b) ** 2).mean()


def sqdist_direct(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Squared L2 distances [nq][n] in float64, direct form sum_i (q_i - x_i)^2."""
    Q = np.asarray(Q, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    out = np.empty((Q.shape[0], X.shape[0]), dtype=np.float64)
    for i in range(Q.shape[0]):
        d = X - Q[i]
        out[i] = np.einsum("nk,nk->n", d, d)
    return out


def topk_by_distance(d: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k smallest distances per row, ties by lower index (stable sort)."""
    return np.argsort(d, axis=1, kind="stable")[:, :k]


def bf16_decode(bits: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> float64 (the upper half of an IEEE single)."""
    b = np.asarray(bits).view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def bf16_encode(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    """OCP FP8 e4m3 bytes -> float64: sign, 4-bit exponent (bias 7), 3-bit mantissa;
    exponent 0 is subnormal (m * 2^-9); 0x7F / 0xFF are NaN."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    e = (c >> 3) & 15
    m = c & 7
    mag = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return np.where(c & 0x80, -mag, mag)


def e4m3_encode(v: np.ndarray) -> np.ndarray:
    """float -> OCP e4m3 bytes by exhaustive nearest search over the 253 finite codes,
    ties to the even code (the one whose mantissa LSB is 0), saturating at +-448; a value
    that rounds to zero keeps its sign (0x00 / 0x80)."""
    v = np.asarray(v, dtype=np.float64)
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = e4m3_decode(codes)
    out = np.empty(v.shape, dtype=np.uint8)
    flat = v.ravel()
    res = out.ravel()
    for i, x in enumerate(flat):
        x = min(max(x, -448.0), 448.0)
        d = np.abs(vals - x)
        best = d.min()
        cand = codes[d == best]
        if len(cand) > 1:   # a tie between two neighbours (or +-0): prefer the even mantissa
            even = [c for c in cand if (c & 1) == 0]
            cand = even if even else cand
        c = int(cand[0])
        if (c & 0x7F) == 0:  # zero magnitude: the sign of the input
            c = 0x80 if np.signbit(x) else 0x00
        res[i] = c
    return out


# ---- binary codes (the paper's unsupervised hashing query, Sec. 2.3) ----

def hash_thresholds(X: np.ndarray) -> np.ndarray:
    """Per column of X [n][dim] the value of 0-based rank (n - 1) // 2 in ascending order
    (the lower median): a full sort per column."""
    X = np.asarray(X, dtype=np.float32)
    return np.sort(X, axis=0)[(X.shape[0] - 1) // 2].astype(np.float32)


def binarize(X: np.ndarray, thr: np.ndarray) -> np.ndarray:
    """uint32 codes [n][dim/32]: bit d (LSB first) = X[d] > thr[d]."""
    bits = np.asarray(X, dtype=np.float32) > np.asarray(thr, dtype=np.float32)[None, :]
    return np.packbits(bits, axis=1, bitorder="little").view("<u4")


def hamming(Qc: np.ndarray, Xc: np.ndarray) -> np.ndarray:
    """float32 [M][N]: number of differing bits of every pair of codes."""
    Q = np.asarray(Qc).view(np.uint8)
    X = np.asarray(Xc).view(np.uint8)
    out = np.empty((Q.shape[0], X.shape[0]), dtype=np.float32)
    for m in range(Q.shape[0]):
        out[m] = np.unpackbits(Q[m][None, :] ^ X, axis=1).sum(axis=1)
    return out


def bihalf_forward(U: np.ndarray) -> np.ndarray:
    """Bi-half layer: per column, the floor(B/2) rows first by (value desc, row asc) -> +1,
    the others -> -1 (same dtype as U)."""
    U = np.asarray(U)
    B, D = U.shape
    out = -np.ones_like(U)
    for d in range(D):
        order = sorted(range(B), key=lambda i: (-float(U[i, d]), i))
        out[order[:B // 2], d] = 1
    return out


def bihalf_backward(U: np.ndarray, Bc: np.ndarray, G: np.ndarray, gamma: float) -> np.ndarray:
    """Straight-through gradient plus the pull towards the code:
    G + gamma * ((U - Bc) / (B * D)), each step rounded in U's dtype."""
    U = np.asarray(U)
    t = U.dtype.type
    B, D = U.shape
    diff = U - np.asarray(Bc, dtype=U.dtype)
    scaled = diff / t(B * D)
    pull = t(gamma) * scaled
    return np.asarray(G, dtype=U.dtype) + pull


# ---- two encoders and the variational head (Sec. 2.3 "Autoencoders") ----

def l2sum_direct(Q1, X1, Q2, X2) -> np.ndarray:
    """L2_T1Gd + L2_FLAIR of two latent sets [nq][n] in float64: sqrt of each direct-form
    squared distance, added."""
    return np.sqrt(sqdist_direct(Q1, X1)) + np.sqrt(sqdist_direct(Q2, X2))


def vae_head(ml: torch.Tensor, eps: torch.Tensor):
    """ml [B][2L] = [mu | logvar] -> (z = mu + exp(logvar / 2) eps,
    KL = (1/B) sum -1/2 (1 + logvar - mu^2 - exp(logvar)))."""
    L = ml.shape[1] // 2
    mu, lv = ml[:, :L], ml[:, L:]
    z = mu + torch.exp(0.5 * lv) * eps
    kl = -0.5 * (1 + lv - mu * mu - torch.exp(lv)).sum() / ml.shape[0]
    return z, kl


def vae_loss(params: dict, x: torch.Tensor, eps: torch.Tensor, beta: float, channels: int, s: int):
    """Reconstruction MSE + beta * KL of the variational autoencoder (float64)."""
    z, kl = vae_head(encode(params, x), eps)
    return mse(decode(params, z, channels, s), x) + beta * kl, kl
