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
