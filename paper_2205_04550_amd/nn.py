"""Convolutional autoencoder on the hand-written HIP kernels of include/tumornn.h.

The paper compresses each tumour with an autoencoder (Sec. 2.3
"Autoencoders", Sec. 2.4 "Implementation"): strided 3-D convolutions
(stride 2, kernel 3) down to a small grid, flatten, a linear layer to the
latent; the decoder mirrors it with strided transposed convolutions; trained
on reconstruction. Here the input is the two masks mean-pooled to half
resolution, the encoder has four stride-2 convolutions (2 -> 8 -> 16 -> 32 ->
64 channels, ReLU) and a linear layer to a 512-d latent; the decoder is a
linear layer (ReLU) and four stride-2 transposed convolutions (ReLU except the
last). Loss: mean squared reconstruction error; optimiser: Adam on FP32
master weights with BF16 working copies of the weights.

Every forward and backward step runs in libtumordb.so; torch only provides
memory, streams and the autograd bookkeeping (torch.autograd.Function).
"""
from __future__ import annotations

import ctypes
import math

import torch

from .binding import LIB, _check

NN_F32, NN_F64, NN_BF16 = 0, 1, 2

_vp, _i32, _i64, _sz, _f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
_SIGS = {
    "nn_meanpool_db": (_i32, [_vp, _vp, _i32, _vp, _i32, _vp]),
    "nn_meanpool_labels": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _vp]),
    "nn_conv3d_s2_fwd": (_i32, [_i32] + [_i32] * 6 + [_vp, _vp, _i32, _vp, _i32, _vp, _vp]),
    "nn_conv3d_s2_bwd_data": (_i32, [_i32] + [_i32] * 6 + [_vp, _vp, _i32, _vp, _i32, _vp, _vp]),
    "nn_conv3d_s2_bwd_weight_ws_bytes": (_sz, [_i32] * 7),
    "nn_conv3d_s2_bwd_weight": (_i32, [_i32] * 7 + [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nn_linear_fwd": (_i32, [_i32] * 4 + [_vp, _vp, _i32, _vp, _i32, _vp, _vp]),
    "nn_linear_bwd_data": (_i32, [_i32] * 4 + [_vp, _vp, _i32, _vp, _vp]),
    "nn_linear_bwd_weight": (_i32, [_i32] * 4 + [_vp, _vp, _vp, _vp, _vp]),
    "nn_channel_sum_ws_bytes": (_sz, [_i32, _i32, _i32, _i64]),
    "nn_channel_sum": (_i32, [_i32, _i32, _i32, _i64, _vp, _vp, _vp, _sz, _vp]),
    "nn_relu_bwd": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp]),
    "nn_mse_ws_bytes": (_sz, [_i32, _i64]),
    "nn_mse_fwd": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nn_mse_bwd": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp, _vp]),
    "nn_adam_step": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _f32, _f32, _f32, _f32, _i32, _vp]),
    "nn_to_bf16": (_i32, [_i64, _vp, _vp, _vp]),
    "nn_bihalf_fwd": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp]),
    "nn_meanpool_db_mask": (_i32, [_vp, _vp, _i32, _i32, _vp, _i32, _vp]),
    "nn_meanpool_labels_mask": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _vp]),
    "nn_pool_conv_labels": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _i32, _vp,
                                   _vp]),
    "nn_pool_conv_planes": (_i32, [_vp, _i64, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp,
                                   _i32, _vp, _vp]),
    "nn_vae_ws_bytes": (_sz, [_i32, _i32, _i32]),
    "nn_vae_head_fwd": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nn_vae_head_bwd": (_i32, [_i32, _i32, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]),
    "nn_bihalf_bwd": (_i32, [_i32, _i32, _i32, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]),
    "nn_pool_conv_labels_bf16": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _i32,
                                        _vp, _vp]),
    "nn_pool_conv_planes_bf16": (_i32, [_vp, _i64, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp,
                                        _vp, _i32, _vp, _vp]),
    "nn_pool_conv_counts_bf16": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _i32,
                                        _vp, _vp]),
    "nn_counts_conv12_bf16": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                     _vp]),
    "nn_conv34_bf16": (_i32, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "nn_conv3d_weights_tapmajor": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "nn_linear_fwd_split": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _i32, _vp, _sz,
                                   _vp]),
    "nn_conv3d_s2_fwd_bf16": (_i32, [_i32] * 6 + [_vp, _vp, _vp, _i32, _i32, _vp, _vp]),
}
for _n, (_r, _a) in _SIGS.items():
    _f = getattr(LIB, _n)
    _f.restype = _r
    _f.argtypes = _a
NN_SYMBOLS = tuple(_SIGS)


def _s() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return NN_F32
    if t.dtype == torch.float64:
        return NN_F64
    raise TypeError(f"activations must be float32 or float64, got {t.dtype}")


def _wdt(w: torch.Tensor) -> int:
    return {torch.bfloat16: NN_BF16, torch.float32: NN_F32, torch.float64: NN_F64}[w.dtype]


def _p(t):
    return None if t is None else t.data_ptr()


def _c(t):
    return t if t.is_contiguous() else t.contiguous()


# ---- pooling ------------------------------------------------------------------------------

def meanpool_db(db, idx: torch.Tensor, dtype=torch.float32, mask: int | None = None) -> torch.Tensor:
    """2x2x2 mean of the masks of database entries idx (int32, device): [B][2][nz/2][ny/2][nx/2],
    or [B][1][...] of one mask (0 FLAIR, 1 T1Gd)."""
    nx, ny, nz = db.dims
    idx = _c(idx.to(torch.int32))
    B = idx.numel()
    out = torch.empty((B, 2 if mask is None else 1, nz // 2, ny // 2, nx // 2), dtype=dtype,
                      device=idx.device)
    if mask is None:
        _check(LIB.nn_meanpool_db(db._h, idx.data_ptr(), B, out.data_ptr(), _dt(out), _s()))
    else:
        _check(LIB.nn_meanpool_db_mask(db._h, idx.data_ptr(), B, mask, out.data_ptr(), _dt(out),
                                       _s()))
    return out


def meanpool_labels(labels: torch.Tensor, dtype=torch.float32, mask: int | None = None) -> torch.Tensor:
    """2x2x2 mean of query labels uint8 [B][nz][ny][nx] (bit0 FLAIR, bit1 T1Gd); one mask with
    mask = 0 / 1."""
    labels = _c(labels)
    if labels.dim() == 3:
        labels = labels[None]
    B, nz, ny, nx = labels.shape
    out = torch.empty((B, 2 if mask is None else 1, nz // 2, ny // 2, nx // 2), dtype=dtype,
                      device=labels.device)
    if mask is None:
        _check(LIB.nn_meanpool_labels(labels.data_ptr(), B, nx, ny, nz, out.data_ptr(), _dt(out),
                                      _s()))
    else:
        _check(LIB.nn_meanpool_labels_mask(labels.data_ptr(), B, nx, ny, nz, mask, out.data_ptr(),
                                           _dt(out), _s()))
    return out


def pool_conv_labels(labels: torch.Tensor, w_bf16: torch.Tensor, bias: torch.Tensor | None,
                     relu: bool = True, mask: int | None = None) -> torch.Tensor:
    """First encoder layer read straight from query labels (forward only): conv(meanpool(labels))
    in one kernel. w_bf16 [Co][Ci][3][3][3] bfloat16 with Ci = 2 (both masks) or 1 (`mask`)."""
    labels = _c(labels)
    if labels.dim() == 3:
        labels = labels[None]
    B, nz, ny, nx = labels.shape
    Co = w_bf16.shape[0]
    assert w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == (2 if mask is None else 1)
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    y = torch.empty((B, Co, nz // 4, ny // 4, nx // 4), dtype=torch.float32, device=labels.device)
    _check(LIB.nn_pool_conv_labels(labels.data_ptr(), B, nx, ny, nz, -1 if mask is None else mask,
                                   Co, w_bf16.data_ptr(), _p(bias), int(relu), y.data_ptr(), _s()))
    return y


def pool_conv_planes(planes: torch.Tensor, dims, w_bf16: torch.Tensor, bias: torch.Tensor | None,
                     relu: bool = True, mask: int | None = None,
                     idx: torch.Tensor | None = None) -> torch.Tensor:
    """pool_conv_labels from packed masks: planes int32 [S][2][Wp] (the database's planes, or
    the queries packed by TumorDB.rerank_pack), samples idx (int32, device) or all S; dims =
    (nx, ny, nz). Equal to pool_conv_labels of the labels that packed to them, bit for bit."""
    nx, ny, nz = dims
    S, two, Wp = planes.shape
    assert two == 2 and planes.is_contiguous()
    B = S if idx is None else idx.numel()
    Co = w_bf16.shape[0]
    assert w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == (2 if mask is None else 1)
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    idx = None if idx is None else _c(idx.to(torch.int32))
    y = torch.empty((B, Co, nz // 4, ny // 4, nx // 4), dtype=torch.float32, device=planes.device)
    _check(LIB.nn_pool_conv_planes(planes.data_ptr(), 2 * Wp, _p(idx), B, nx, ny, nz,
                                   -1 if mask is None else mask, Co, w_bf16.data_ptr(), _p(bias),
                                   int(relu), y.data_ptr(), _s()))
    return y


# ---- BF16 inference forward -----------------------------------------------------------------
# Activations bfloat16 channels-last [B][D][H][W][C]; each layer rounds its FP32 result to the
# nearest bfloat16. Forward only (no autograd).

def pool_conv_labels_bf16(labels: torch.Tensor, w_bf16: torch.Tensor, bias: torch.Tensor | None,
                          relu: bool = True, mask: int | None = None) -> torch.Tensor:
    """pool_conv_labels with a bfloat16 channels-last output [B][nz/4][ny/4][nx/4][Co]."""
    labels = _c(labels)
    if labels.dim() == 3:
        labels = labels[None]
    B, nz, ny, nx = labels.shape
    Co = w_bf16.shape[0]
    assert w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == (2 if mask is None else 1)
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    y = torch.empty((B, nz // 4, ny // 4, nx // 4, Co), dtype=torch.bfloat16, device=labels.device)
    _check(LIB.nn_pool_conv_labels_bf16(labels.data_ptr(), B, nx, ny, nz,
                                        -1 if mask is None else mask, Co, w_bf16.data_ptr(),
                                        _p(bias), int(relu), y.data_ptr(), _s()))
    return y


def pool_conv_planes_bf16(planes: torch.Tensor, dims, w_bf16: torch.Tensor,
                          bias: torch.Tensor | None, relu: bool = True, mask: int | None = None,
                          idx: torch.Tensor | None = None) -> torch.Tensor:
    """pool_conv_planes with the output of pool_conv_labels_bf16."""
    nx, ny, nz = dims
    S, two, Wp = planes.shape
    assert two == 2 and planes.is_contiguous()
    B = S if idx is None else idx.numel()
    Co = w_bf16.shape[0]
    assert w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == (2 if mask is None else 1)
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    idx = None if idx is None else _c(idx.to(torch.int32))
    y = torch.empty((B, nz // 4, ny // 4, nx // 4, Co), dtype=torch.bfloat16, device=planes.device)
    _check(LIB.nn_pool_conv_planes_bf16(planes.data_ptr(), 2 * Wp, _p(idx), B, nx, ny, nz,
                                        -1 if mask is None else mask, Co, w_bf16.data_ptr(),
                                        _p(bias), int(relu), y.data_ptr(), _s()))
    return y


def pool_conv_counts_bf16(counts: torch.Tensor, w_bf16: torch.Tensor, bias: torch.Tensor | None,
                          relu: bool = True, mask: int | None = None) -> torch.Tensor:
    """pool_conv_labels_bf16 from the pooled counts uint8 [B][nz/2][ny/2][nx/2] that
    TumorDB.rerank_pack_pool writes; equal to it bit for bit for the labels they came from."""
    counts = _c(counts)
    B, pz, py, px = counts.shape
    nz, ny, nx = 2 * pz, 2 * py, 2 * px
    Co = w_bf16.shape[0]
    assert counts.dtype == torch.uint8
    assert w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == (2 if mask is None else 1)
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    y = torch.empty((B, nz // 4, ny // 4, nx // 4, Co), dtype=torch.bfloat16, device=counts.device)
    _check(LIB.nn_pool_conv_counts_bf16(counts.data_ptr(), B, nx, ny, nz,
                                        -1 if mask is None else mask, Co, w_bf16.data_ptr(),
                                        _p(bias), int(relu), y.data_ptr(), _s()))
    return y


def counts_conv12_bf16(counts: torch.Tensor, w1_bf16: torch.Tensor, b1: torch.Tensor | None,
                       w2_tm: torch.Tensor, b2: torch.Tensor | None,
                       mask: int | None = None) -> torch.Tensor:
    """The encoder's first two layers (8 then 16 channels, ReLU) from pooled counts uint8
    [B][nz/2][ny/2][nx/2] in one kernel: conv3d_bf16(pool_conv_counts_bf16(...)) bit for bit,
    bfloat16 channels-last [B][nz/8][ny/8][nx/8][16]."""
    counts = _c(counts)
    B, pz, py, px = counts.shape
    nz, ny, nx = 2 * pz, 2 * py, 2 * px
    assert counts.dtype == torch.uint8
    assert w1_bf16.dtype == torch.bfloat16 and w1_bf16.shape[:2] == (8, 2 if mask is None else 1)
    assert w2_tm.dtype == torch.bfloat16 and tuple(w2_tm.shape) == (16, 28, 8)
    w1_bf16, w2_tm = _c(w1_bf16), _c(w2_tm)
    b1 = None if b1 is None else _c(b1.detach())
    b2 = None if b2 is None else _c(b2.detach())
    y = torch.empty((B, nz // 8, ny // 8, nx // 8, 16), dtype=torch.bfloat16, device=counts.device)
    _check(LIB.nn_counts_conv12_bf16(counts.data_ptr(), B, nx, ny, nz, -1 if mask is None else mask,
                                     w1_bf16.data_ptr(), _p(b1), w2_tm.data_ptr(), _p(b2),
                                     y.data_ptr(), _s()))
    return y


def conv34_bf16(x: torch.Tensor, w3_tm: torch.Tensor, b3: torch.Tensor | None,
                w4_tm: torch.Tensor, b4: torch.Tensor | None) -> torch.Tensor:
    """The third and fourth layers (ReLU; 16 -> 32 -> 64 channels) of bfloat16 channels-last
    x [B][16][16][16][16] in one kernel: conv3d_bf16 twice (the second with float output),
    bit for bit; float [B][64][4][4][4]."""
    x = _c(x)
    assert x.dtype == torch.bfloat16 and tuple(x.shape[1:]) == (16, 16, 16, 16)
    assert tuple(w3_tm.shape) == (32, 28, 16) and tuple(w4_tm.shape) == (64, 28, 32)
    b3 = None if b3 is None else _c(b3.detach())
    b4 = None if b4 is None else _c(b4.detach())
    y = torch.empty((x.shape[0], 64, 4, 4, 4), dtype=torch.float32, device=x.device)
    _check(LIB.nn_conv34_bf16(x.shape[0], x.data_ptr(), _c(w3_tm).data_ptr(), _p(b3),
                              _c(w4_tm).data_ptr(), _p(b4), y.data_ptr(), _s()))
    return y


def linear_split(x: torch.Tensor, w_bf16: torch.Tensor, bias: torch.Tensor | None,
                 relu: bool = False, splits: int = 4) -> torch.Tensor:
    """Forward-only linear layer (float x [B][In], bfloat16 weights [Out][In]) with K split into
    `splits` slices summed in a fixed order: the encoder head for a batch of queries."""
    x = _c(x)
    B, In = x.shape
    Out = w_bf16.shape[0]
    assert x.dtype == torch.float32 and w_bf16.dtype == torch.bfloat16 and w_bf16.shape[1] == In
    w_bf16 = _c(w_bf16)
    bias = None if bias is None else _c(bias.detach())
    y = torch.empty((B, Out), dtype=torch.float32, device=x.device)
    ws = torch.empty(splits * B * Out, dtype=torch.float32, device=x.device)
    _check(LIB.nn_linear_fwd_split(B, In, Out, x.data_ptr(), w_bf16.data_ptr(), _p(bias),
                                   int(relu), y.data_ptr(), splits, ws.data_ptr(),
                                   ws.numel() * 4, _s()))
    return y


def conv_weights_tapmajor(w_bf16: torch.Tensor) -> torch.Tensor:
    """[Co][Ci][3][3][3] bfloat16 -> [Co][28][Ci] (tap-major, tap 27 zero) for conv3d_bf16."""
    assert w_bf16.dtype == torch.bfloat16
    Co, Ci = w_bf16.shape[:2]
    out = torch.empty((Co, 28, Ci), dtype=torch.bfloat16, device=w_bf16.device)
    _check(LIB.nn_conv3d_weights_tapmajor(_c(w_bf16).data_ptr(), Co, Ci, out.data_ptr(), _s()))
    return out


def conv3d_bf16(x: torch.Tensor, w_tm: torch.Tensor, bias: torch.Tensor | None, relu: bool = True,
                out_f32: bool = False) -> torch.Tensor:
    """Stride-2 convolution of bfloat16 channels-last x [B][D][H][W][Ci] with tap-major weights
    w_tm [Co][28][Ci]: bfloat16 [B][D/2][H/2][W/2][Co], or float [B][Co][D/2][H/2][W/2]."""
    x = _c(x)
    assert x.dtype == torch.bfloat16 and w_tm.dtype == torch.bfloat16
    B, D, H, W, Ci = x.shape
    Co = w_tm.shape[0]
    bias = None if bias is None else _c(bias.detach())
    if out_f32:
        y = torch.empty((B, Co, D // 2, H // 2, W // 2), dtype=torch.float32, device=x.device)
    else:
        y = torch.empty((B, D // 2, H // 2, W // 2, Co), dtype=torch.bfloat16, device=x.device)
    _check(LIB.nn_conv3d_s2_fwd_bf16(B, Ci, Co, D, H, W, x.data_ptr(), _c(w_tm).data_ptr(),
                                     _p(bias), int(relu), int(out_f32), y.data_ptr(), _s()))
    return y


# ---- autograd functions ---------------------------------------------------------------------

class Conv3dS2(torch.autograd.Function):
    """y = act(conv3d(x, w, b, stride 2, padding 1)); w_compute is the weight copy used."""

    @staticmethod
    def forward(ctx, x, w, b, w_compute, relu: bool):
        x = _c(x)
        B, Ci, D, H, W = x.shape
        Co = w.shape[0]
        y = torch.empty((B, Co, D // 2, H // 2, W // 2), dtype=x.dtype, device=x.device)
        _check(LIB.nn_conv3d_s2_fwd(_dt(x), B, Ci, Co, D, H, W, x.data_ptr(), w_compute.data_ptr(),
                                    _wdt(w_compute), _p(b), int(relu), y.data_ptr(), _s()))
        ctx.save_for_backward(x, w_compute, y)
        ctx.relu = relu
        ctx.has_bias = b is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, wc, y = ctx.saved_tensors
        B, Ci, D, H, W = x.shape
        Co = wc.shape[0]
        gy = _c(gy)
        if ctx.relu:
            g = torch.empty_like(gy)
            _check(LIB.nn_relu_bwd(_dt(gy), gy.numel(), y.data_ptr(), gy.data_ptr(), g.data_ptr(), _s()))
        else:
            g = gy
        dx = None
        if ctx.needs_input_grad[0]:
            dx = torch.empty_like(x)
            _check(LIB.nn_conv3d_s2_bwd_data(_dt(x), B, Ci, Co, D, H, W, g.data_ptr(), wc.data_ptr(),
                                             _wdt(wc), None, 0, dx.data_ptr(), _s()))
        dw = torch.empty((Co, Ci, 3, 3, 3), dtype=x.dtype, device=x.device)
        db_ = torch.empty(Co, dtype=x.dtype, device=x.device) if ctx.has_bias else None
        nb = LIB.nn_conv3d_s2_bwd_weight_ws_bytes(_dt(x), B, Ci, Co, D, H, W)
        ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
        _check(LIB.nn_conv3d_s2_bwd_weight(_dt(x), B, Ci, Co, D, H, W, x.data_ptr(), g.data_ptr(),
                                           dw.data_ptr(), _p(db_), ws.data_ptr(), nb, _s()))
        return dx, dw, db_, None, None


class ConvT3dS2(torch.autograd.Function):
    """y = act(conv_transpose3d(x, w, b, stride 2, padding 1, output_padding 1)).

    w has the transposed-convolution layout [Cin][Cout][3][3][3]; the map is
    the adjoint of the stride-2 convolution with weight w viewed as
    [Co = Cin][Ci = Cout].
    """

    @staticmethod
    def forward(ctx, x, w, b, w_compute, relu: bool):
        x = _c(x)
        B, Cin, d, h, wd = x.shape
        Cout = w.shape[1]
        D, H, W = 2 * d, 2 * h, 2 * wd
        y = torch.empty((B, Cout, D, H, W), dtype=x.dtype, device=x.device)
        _check(LIB.nn_conv3d_s2_bwd_data(_dt(x), B, Cout, Cin, D, H, W, x.data_ptr(),
                                         w_compute.data_ptr(), _wdt(w_compute), _p(b), int(relu),
                                         y.data_ptr(), _s()))
        ctx.save_for_backward(x, w_compute, y)
        ctx.relu = relu
        ctx.has_bias = b is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, wc, y = ctx.saved_tensors
        B, Cin, d, h, wd = x.shape
        Cout = wc.shape[1]
        D, H, W = 2 * d, 2 * h, 2 * wd
        gy = _c(gy)
        if ctx.relu:
            g = torch.empty_like(gy)
            _check(LIB.nn_relu_bwd(_dt(gy), gy.numel(), y.data_ptr(), gy.data_ptr(), g.data_ptr(), _s()))
        else:
            g = gy
        dx = None
        if ctx.needs_input_grad[0]:
            dx = torch.empty_like(x)
            _check(LIB.nn_conv3d_s2_fwd(_dt(x), B, Cout, Cin, D, H, W, g.data_ptr(), wc.data_ptr(),
                                        _wdt(wc), None, 0, dx.data_ptr(), _s()))
        dw = torch.empty((Cin, Cout, 3, 3, 3), dtype=x.dtype, device=x.device)
        nb = LIB.nn_conv3d_s2_bwd_weight_ws_bytes(_dt(x), B, Cout, Cin, D, H, W)
        ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
        _check(LIB.nn_conv3d_s2_bwd_weight(_dt(x), B, Cout, Cin, D, H, W, g.data_ptr(), x.data_ptr(),
                                           dw.data_ptr(), None, ws.data_ptr(), nb, _s()))
        db_ = None
        if ctx.has_bias:
            db_ = torch.empty(Cout, dtype=x.dtype, device=x.device)
            nbs = LIB.nn_channel_sum_ws_bytes(_dt(x), B, Cout, D * H * W)
            wss = torch.empty(nbs, dtype=torch.uint8, device=x.device)
            _check(LIB.nn_channel_sum(_dt(x), B, Cout, D * H * W, g.data_ptr(), db_.data_ptr(),
                                      wss.data_ptr(), nbs, _s()))
        return dx, dw, db_, None, None


class Linear(torch.autograd.Function):
    """y = act(x w^T + b), x [B][In], w [Out][In]."""

    @staticmethod
    def forward(ctx, x, w, b, w_compute, relu: bool):
        x = _c(x)
        B, In = x.shape
        Out = w.shape[0]
        y = torch.empty((B, Out), dtype=x.dtype, device=x.device)
        _check(LIB.nn_linear_fwd(_dt(x), B, In, Out, x.data_ptr(), w_compute.data_ptr(),
                                 _wdt(w_compute), _p(b), int(relu), y.data_ptr(), _s()))
        ctx.save_for_backward(x, w_compute, y)
        ctx.relu = relu
        ctx.has_bias = b is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, wc, y = ctx.saved_tensors
        B, In = x.shape
        Out = wc.shape[0]
        gy = _c(gy)
        if ctx.relu:
            g = torch.empty_like(gy)
            _check(LIB.nn_relu_bwd(_dt(gy), gy.numel(), y.data_ptr(), gy.data_ptr(), g.data_ptr(), _s()))
        else:
            g = gy
        dx = None
        if ctx.needs_input_grad[0]:
            dx = torch.empty_like(x)
            _check(LIB.nn_linear_bwd_data(_dt(x), B, In, Out, g.data_ptr(), wc.data_ptr(), _wdt(wc),
                                          dx.data_ptr(), _s()))
        dw = torch.empty((Out, In), dtype=x.dtype, device=x.device)
        db_ = torch.empty(Out, dtype=x.dtype, device=x.device) if ctx.has_bias else None
        _check(LIB.nn_linear_bwd_weight(_dt(x), B, In, Out, x.data_ptr(), g.data_ptr(), dw.data_ptr(),
                                        _p(db_), _s()))
        return dx, dw, db_, None, None


class MSE(torch.autograd.Function):
    """mean((a - b)^2); b is the target (no gradient)."""

    @staticmethod
    def forward(ctx, a, b):
        a, b = _c(a), _c(b)
        n = a.numel()
        loss = torch.empty((), dtype=a.dtype, device=a.device)
        nb = LIB.nn_mse_ws_bytes(_dt(a), n)
        ws = torch.empty(nb, dtype=torch.uint8, device=a.device)
        _check(LIB.nn_mse_fwd(_dt(a), n, a.data_ptr(), b.data_ptr(), loss.data_ptr(), ws.data_ptr(),
                              nb, _s()))
        ctx.save_for_backward(a, b)
        return loss

    @staticmethod
    def backward(ctx, gl):
        a, b = ctx.saved_tensors
        gl = _c(gl.to(a.dtype))
        da = torch.empty_like(a)
        _check(LIB.nn_mse_bwd(_dt(a), a.numel(), a.data_ptr(), b.data_ptr(), gl.data_ptr(),
                              da.data_ptr(), _s()))
        return da, None


class BiHalf(torch.autograd.Function):
    """The Bi-half hash layer (Sec. 2.3, unsupervised hashing): per coordinate the larger half
    of the batch -> +1, the rest -> -1; backward passes the gradient straight through plus
    gamma * (U - B) / (B * D)."""

    @staticmethod
    def forward(ctx, u, gamma):
        u = _c(u)
        B, D = u.shape
        b = torch.empty_like(u)
        _check(LIB.nn_bihalf_fwd(_dt(u), B, D, u.data_ptr(), b.data_ptr(), _s()))
        ctx.save_for_backward(u, b)
        ctx.gamma = float(gamma)
        return b

    @staticmethod
    def backward(ctx, g):
        u, b = ctx.saved_tensors
        g = _c(g.to(u.dtype))
        du = torch.empty_like(u)
        B, D = u.shape
        _check(LIB.nn_bihalf_bwd(_dt(u), B, D, ctx.gamma, u.data_ptr(), b.data_ptr(), g.data_ptr(),
                                 du.data_ptr(), _s()))
        return du, None


class VaeHead(torch.autograd.Function):
    """z = mu + exp(logvar / 2) * eps from ML = [mu | logvar] (one linear layer of 2L outputs);
    the backward also carries beta * KL, whose value is left in ctx-free `kl_out`."""

    @staticmethod
    def forward(ctx, ml, eps, beta, kl_out):
        ml, eps = _c(ml), _c(eps)
        B, L2 = ml.shape
        L = L2 // 2
        z = torch.empty((B, L), dtype=ml.dtype, device=ml.device)
        nb = LIB.nn_vae_ws_bytes(_dt(ml), B, L)
        ws = torch.empty(nb, dtype=torch.uint8, device=ml.device)
        _check(LIB.nn_vae_head_fwd(_dt(ml), B, L, ml.data_ptr(), eps.data_ptr(), z.data_ptr(),
                                   kl_out.data_ptr(), ws.data_ptr(), nb, _s()))
        ctx.save_for_backward(ml, eps)
        ctx.beta = float(beta)
        return z

    @staticmethod
    def backward(ctx, dz):
        ml, eps = ctx.saved_tensors
        dz = _c(dz.to(ml.dtype))
        B, L2 = ml.shape
        dml = torch.empty_like(ml)
        _check(LIB.nn_vae_head_bwd(_dt(ml), B, L2 // 2, ctx.beta, ml.data_ptr(), eps.data_ptr(),
                                   dz.data_ptr(), dml.data_ptr(), _s()))
        return dml, None, None, None


# ---- model ----------------------------------------------------------------------------------

class AutoEncoder:
    """Encoder 2->8->16->32->64 stride-2 convolutions + linear to `latent`, mirrored decoder.

    dtype float32: BF16 working weights, FP32 master weights, activations and
    biases. dtype float64: every weight in double (for gradient checks).
    """

    def __init__(self, grid: int = 64, channels=(2, 8, 16, 32, 64), latent: int = 512,
                 dtype=torch.float32, device="cuda", seed: int = 0, hash_gamma: float | None = None,
                 vae_beta: float | None = None):
        assert grid % 16 == 0
        assert hash_gamma is None or vae_beta is None
        self.grid, self.channels, self.latent = grid, tuple(channels), latent
        # With hash_gamma the decoder reads the Bi-half codes of the latent (the paper's
        # hashing autoencoder); with vae_beta the encoder's last layer gives mean and
        # log-variance (the paper's VAE) and training adds vae_beta * KL; otherwise the
        # decoder reads the latent itself.
        self.hash_gamma = hash_gamma
        self.vae_beta = vae_beta
        self.kl = None          # KL of the last variational forward (device scalar)
        self._eps_gen = None
        self.dtype = dtype
        self.bf16 = dtype == torch.float32
        g = torch.Generator().manual_seed(seed)
        s = grid // 16
        self.flat = channels[-1] * s ** 3
        self.params = {}

        def uni(shape, fan_in):
            bound = math.sqrt(6.0 / fan_in)   # He-uniform for ReLU layers
            return ((torch.rand(shape, generator=g, dtype=torch.float64) * 2 - 1) * bound)

        for i in range(4):
            ci, co = channels[i], channels[i + 1]
            self.params[f"enc{i}.w"] = uni((co, ci, 3, 3, 3), ci * 27)
            self.params[f"enc{i}.b"] = torch.zeros(co, dtype=torch.float64)
        heads = 2 if vae_beta is not None else 1   # [mu | logvar] rows for the VAE
        self.params["enc_fc.w"] = uni((heads * latent, self.flat), self.flat)
        self.params["enc_fc.b"] = torch.zeros(heads * latent, dtype=torch.float64)
        self.params["dec_fc.w"] = uni((self.flat, latent), latent)
        self.params["dec_fc.b"] = torch.zeros(self.flat, dtype=torch.float64)
        for i in reversed(range(4)):
            ci, co = channels[i + 1], channels[i]       # transposed conv: Cin -> Cout
            self.params[f"dec{i}.w"] = uni((ci, co, 3, 3, 3), ci * 27)
            self.params[f"dec{i}.b"] = torch.zeros(co, dtype=torch.float64)
        for k in self.params:
            self.params[k] = self.params[k].to(device=device, dtype=dtype).requires_grad_(True)
        self.work = {}
        # Version of the working weights (refresh_working_weights and every Adam step bump it),
        # and the version the tap-major copies of the BF16 forward were made from.
        self.work_version, self._tm_version, self.work_tm = 0, -1, {}
        self.refresh_working_weights()

    def refresh_working_weights(self) -> None:
        """BF16 copies (round to nearest even) of the weight tensors, or the weights themselves."""
        for k, p in self.params.items():
            if not k.endswith(".w"):
                continue
            if self.bf16:
                wb = self.work.get(k)
                if wb is None:
                    wb = torch.empty(p.shape, dtype=torch.bfloat16, device=p.device)
                    self.work[k] = wb
                _check(LIB.nn_to_bf16(p.numel(), p.data_ptr(), wb.data_ptr(), _s()))
            else:
                self.work[k] = p.detach()
        self.work_version += 1

    def _w(self, name):
        return self.params[name + ".w"], self.params[name + ".b"], self.work[name + ".w"]

    def _features(self, x: torch.Tensor) -> torch.Tensor:
        h = x
        for i in range(4):
            w, b, wc = self._w(f"enc{i}")
            h = Conv3dS2.apply(h, w, b, wc, True)
        return h.reshape(h.shape[0], -1)

    def encode(self, x: torch.Tensor) -> torch.Tensor:
        """The latent (for the VAE: the mean, from the first `latent` rows of the head)."""
        return self._head(self._features(x))

    def encode_labels(self, labels: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """encode(meanpool_labels(labels, mask=mask)) for inference, the pooling fused into the
        first convolution when the shapes allow it (BF16 weights, nx % 128 == 0)."""
        nz, ny, nx = labels.shape[-3:]
        if not (self.bf16 and nx % 128 == 0 and ny % 4 == 0 and nz % 4 == 0
                and self.channels[1] <= 16):
            return self.encode(meanpool_labels(labels, mask=mask))
        return self.encode_after_first(self.first_layer_labels(labels, mask))

    def first_layer_labels(self, labels: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """The fused first layer of encode_labels alone (pooling + convolution from the label
        bytes), so a caller can start other work between it and encode_after_first."""
        with torch.no_grad():
            w, b, wc = self._w("enc0")
            return pool_conv_labels(labels, wc, b, True, mask)

    def encode_after_first(self, h: torch.Tensor) -> torch.Tensor:
        """The rest of the encoder after the first layer's output h."""
        with torch.no_grad():
            for i in range(1, 4):
                w, b, wc = self._w(f"enc{i}")
                h = Conv3dS2.apply(h, w, b, wc, True)
            return self._head(h.reshape(h.shape[0], -1))

    def encode_planes(self, planes: torch.Tensor, dims, idx: torch.Tensor | None = None,
                      mask: int | None = None) -> torch.Tensor:
        """encode_labels from packed masks (planes int32 [S][2][Wp], samples idx or all): the
        first layer pools the bit planes (pool_conv_planes); needs the fused path's shapes."""
        nx, ny, nz = dims
        assert self.bf16 and nx % 128 == 0 and ny % 4 == 0 and nz % 4 == 0 and self.channels[1] <= 16
        with torch.no_grad():
            w, b, wc = self._w("enc0")
            h = pool_conv_planes(planes, dims, wc, b, True, mask, idx)
            for i in range(1, 4):
                w, b, wc = self._w(f"enc{i}")
                h = Conv3dS2.apply(h, w, b, wc, True)
            return self._head(h.reshape(h.shape[0], -1))

    # ---- BF16 inference forward: bfloat16 channels-last activations, each layer's FP32 result
    # rounded to bfloat16 (a different numerics contract from encode; see conv3d_bf16).

    def bf16_inference_ok(self, dims) -> bool:
        """Whether the BF16 forward covers this model and mask grid (nx, ny, nz)."""
        nx, ny, nz = dims
        return (self.bf16 and tuple(self.channels[1:]) == (8, 16, 32, 64)
                and nx % 128 == 0 and ny % 128 == 0 and nz % 128 == 0)

    def first_layer_labels_bf16(self, labels: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """The fused first layer from label bytes, bfloat16 channels-last output."""
        with torch.no_grad():
            w, b, wc = self._w("enc0")
            return pool_conv_labels_bf16(labels, wc, b, True, mask)

    def first_layer_counts_bf16(self, counts: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """first_layer_labels_bf16 from pooled counts (TumorDB.rerank_pack_pool), bit for bit."""
        with torch.no_grad():
            w, b, wc = self._w("enc0")
            return pool_conv_counts_bf16(counts, wc, b, True, mask)

    def _tapmajor(self) -> dict:
        """Tap-major copies of the later convolutions' working weights, remade whenever the
        working weights changed (training updates them in place)."""
        if self._tm_version != self.work_version:
            self.work_tm = {f"enc{i}": conv_weights_tapmajor(self.work[f"enc{i}.w"])
                            for i in range(1, 4)}
            self._tm_version = self.work_version
        return self.work_tm

    def encode_after_first_bf16(self, h: torch.Tensor, first: int = 1) -> torch.Tensor:
        """The convolutions from layer `first` on (BF16 matrix cores), then the head (float)."""
        with torch.no_grad():
            tm = self._tapmajor()
            if first == 2 and tuple(h.shape[1:]) == (16, 16, 16, 16):   # layers 3 and 4 fused
                _, b3, _ = self._w("enc2")
                _, b4, _ = self._w("enc3")
                h = conv34_bf16(h, tm["enc2"], b3, tm["enc3"], b4)
                first = 4
            for i in range(first, 4):
                w, b, wc = self._w(f"enc{i}")
                h = conv3d_bf16(h, tm[f"enc{i}"], b, True, out_f32=(i == 3))
            w, b, wc = self._w("enc_fc")
            L = self.latent
            return linear_split(h.reshape(h.shape[0], -1), wc[:L], b[:L])

    def encode_labels_bf16(self, labels: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """Latents of query labels [B][nz][ny][nx] by the BF16 forward."""
        nz, ny, nx = labels.shape[-3:]
        assert self.bf16_inference_ok((nx, ny, nz))
        return self.encode_after_first_bf16(self.first_layer_labels_bf16(labels, mask))

    def encode_counts_bf16(self, counts: torch.Tensor, mask: int | None = None) -> torch.Tensor:
        """encode_labels_bf16 from pooled counts [B][nz/2][ny/2][nx/2], bit for bit (the first
        two layers in one kernel)."""
        pz, py, px = counts.shape[-3:]
        assert self.bf16_inference_ok((2 * px, 2 * py, 2 * pz))
        with torch.no_grad():
            _, b1, wc1 = self._w("enc0")
            _, b2, _ = self._w("enc1")
            h = counts_conv12_bf16(counts, wc1, b1, self._tapmajor()["enc1"], b2, mask)
        return self.encode_after_first_bf16(h, first=2)

    def encode_planes_bf16(self, planes: torch.Tensor, dims, idx: torch.Tensor | None = None,
                           mask: int | None = None) -> torch.Tensor:
        """encode_labels_bf16 from packed masks (the database's planes, or packed queries);
        equal to it bit for bit for the labels that packed to these masks."""
        assert self.bf16_inference_ok(dims)
        with torch.no_grad():
            w, b, wc = self._w("enc0")
            h = pool_conv_planes_bf16(planes, dims, wc, b, True, mask, idx)
        return self.encode_after_first_bf16(h)

    def _head(self, h: torch.Tensor) -> torch.Tensor:
        w, b, wc = self._w("enc_fc")
        if self.vae_beta is None:
            return Linear.apply(h, w, b, wc, False)
        L = self.latent
        return Linear.apply(h, w[:L], b[:L], wc[:L], False)

    def decode(self, z: torch.Tensor) -> torch.Tensor:
        w, b, wc = self._w("dec_fc")
        h = Linear.apply(z, w, b, wc, True)
        s = self.grid // 16
        h = h.reshape(h.shape[0], self.channels[-1], s, s, s)
        for i in reversed(range(4)):
            w, b, wc = self._w(f"dec{i}")
            h = ConvT3dS2.apply(h, w, b, wc, i != 0)
        return h

    def forward(self, x: torch.Tensor, eps: torch.Tensor | None = None) -> torch.Tensor:
        if self.vae_beta is not None:
            h = self._features(x)
            w, b, wc = self._w("enc_fc")
            ml = Linear.apply(h, w, b, wc, False)
            if eps is None:
                if self._eps_gen is None:
                    self._eps_gen = torch.Generator(device=x.device).manual_seed(12345)
                eps = torch.randn((x.shape[0], self.latent), generator=self._eps_gen,
                                  dtype=x.dtype, device=x.device)
            self.kl = torch.empty((), dtype=x.dtype, device=x.device)
            z = VaeHead.apply(ml, eps, self.vae_beta, self.kl)
            return self.decode(z)
        z = self.encode(x)
        if self.hash_gamma is not None:
            z = BiHalf.apply(z, self.hash_gamma)
        return self.decode(z)

    def loss(self, x: torch.Tensor, eps: torch.Tensor | None = None) -> torch.Tensor:
        """Reconstruction MSE. For the VAE the backward also applies vae_beta * KL (its value
        is in self.kl after the call)."""
        return MSE.apply(self.forward(x, eps), x)

    def n_params(self) -> int:
        return sum(p.numel() for p in self.params.values())


class Adam:
    """Adam on the FP32 master weights; refreshes the BF16 working copies in the same kernel."""

    def __init__(self, model: AutoEncoder, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        assert model.dtype == torch.float32
        self.model, self.lr, self.b1, self.b2, self.eps = model, lr, betas[0], betas[1], eps
        self.m = {k: torch.zeros_like(p, requires_grad=False) for k, p in model.params.items()}
        self.v = {k: torch.zeros_like(p, requires_grad=False) for k, p in model.params.items()}
        self.t = 0

    def step(self) -> None:
        self.t += 1
        for k, p in self.model.params.items():
            if p.grad is None:
                continue
            wb = self.model.work.get(k) if (self.model.bf16 and k.endswith(".w")) else None
            _check(LIB.nn_adam_step(p.numel(), p.data_ptr(), self.m[k].data_ptr(), self.v[k].data_ptr(),
                                    p.grad.data_ptr(), _p(wb), self.lr, self.b1, self.b2, self.eps,
                                    self.t, _s()))
            p.grad = None
        self.model.work_version += 1


def train_step(model: AutoEncoder, opt: Adam, x: torch.Tensor) -> torch.Tensor:
    """One step: forward, MSE against the input, backward, Adam. Returns the loss (device)."""
    loss = model.loss(x)
    loss.backward()
    opt.step()
    return loss.detach()
