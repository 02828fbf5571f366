"""Pins of the embedding-path oracle (CPU, float64) against closed forms and identities."""
import numpy as np
import torch

from oracle import encoder as E


def test_meanpool_closed_forms():
    lab = np.zeros((1, 4, 4, 8), dtype=np.uint8)
    lab[0, 1, 2, 5] = 1          # one FLAIR voxel -> 1/8 in block (0, 1, 2)
    lab[0, 2:4, 0:2, 0:2] = 3    # a full 2x2x2 block of both masks -> 1
    out = E.meanpool(lab)
    assert out.shape == (1, 2, 2, 2, 4)
    assert out[0, 0, 0, 1, 2] == 0.125
    assert out[0, 0, 1, 0, 0] == 1.0 and out[0, 1, 1, 0, 0] == 1.0
    assert out[0, 1, 0, 1, 2] == 0.0
    rng = np.random.default_rng(0)
    lab = rng.integers(0, 4, size=(2, 6, 8, 32), dtype=np.uint8)
    out = E.meanpool(lab)
    for m in range(2):
        assert out[:, m].sum() * 8 == ((lab >> m) & 1).sum()
    assert set(np.unique(out * 8)) <= set(range(9))


def test_conv_with_centre_delta_is_strided_copy():
    torch.manual_seed(0)
    x = torch.randn(2, 3, 8, 6, 4, dtype=torch.float64)
    w = torch.zeros(3, 3, 3, 3, 3, dtype=torch.float64)
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0                     # centre tap -> input voxel 2o
    y = E.conv(x, w, None, False)
    assert torch.equal(y, x[:, :, ::2, ::2, ::2])
    w2 = torch.zeros_like(w)
    for c in range(3):
        w2[c, c, 2, 2, 2] = 1.0                    # last tap -> input voxel 2o + 1
    y2 = E.conv(x, w2, None, False)
    assert torch.equal(y2, x[:, :, 1::2, 1::2, 1::2])


def test_transposed_conv_is_the_adjoint():
    torch.manual_seed(1)
    x = torch.randn(2, 4, 8, 8, 6, dtype=torch.float64)
    w = torch.randn(5, 4, 3, 3, 3, dtype=torch.float64)      # conv: 4 -> 5 channels
    y = torch.randn(2, 5, 4, 4, 3, dtype=torch.float64)
    lhs = (E.conv(x, w, None, False) * y).sum()
    rhs = (x * E.conv_t(y, w, None, False)).sum()               # same tensor as [Cin][Cout]
    assert abs(float(lhs - rhs)) <= 1e-10 * abs(float(lhs))
    assert E.conv_t(y, w, None, False).shape == x.shape


def test_linear_identity_and_relu():
    z = torch.randn(3, 7, dtype=torch.float64)
    assert torch.equal(torch.nn.functional.linear(z, torch.eye(7, dtype=torch.float64)), z)
    w = torch.zeros(2, 2, 3, 3, 3, dtype=torch.float64)
    w[0, 0, 1, 1, 1] = 1.0
    w[1, 1, 1, 1, 1] = 1.0
    # A 2x2x2 grid: the centre tap of output voxel 0 reads input voxel 0.
    x = torch.zeros(1, 2, 2, 2, 2, dtype=torch.float64)
    x[0, 0, 0, 0, 0], x[0, 1, 0, 0, 0] = -1.0, 2.0
    y = E.conv(x, w, None, True)
    assert y.shape == (1, 2, 1, 1, 1)
    assert float(y[0, 0]) == 0.0 and float(y[0, 1]) == 2.0


def test_distance_forms():
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((4, 16))
    X = np.concatenate([Q[:2], rng.standard_normal((5, 16))])
    d = E.sqdist_direct(Q, X)
    assert d[0, 0] == 0.0 and d[1, 1] == 0.0
    e = np.eye(16)
    assert E.sqdist_direct(e[:1], e[1:2])[0, 0] == 2.0
    expanded = (Q ** 2).sum(1)[:, None] + (X ** 2).sum(1)[None, :] - 2 * Q @ X.T
    assert np.allclose(expanded, d, atol=1e-12)
    top = E.topk_by_distance(np.array([[3.0, 1.0, 1.0, 0.5]]), 3)
    assert top.tolist() == [[3, 1, 2]]


def test_mse_gradient_closed_form():
    a = torch.randn(3, 5, dtype=torch.float64, requires_grad=True)
    b = torch.randn(3, 5, dtype=torch.float64)
    E.mse(a, b).backward()
    assert torch.allclose(a.grad, 2 * (a.detach() - b) / a.numel(), rtol=0, atol=1e-15)


def test_e4m3_format_pins():
    # Values fixed by the OCP e4m3 definition (bias 7, 3 mantissa bits, max 448, no inf).
    assert E.e4m3_decode(np.array([0x38, 0x40, 0x7E, 0x08, 0x01, 0xC0, 0x00])).tolist() == \
        [1.0, 2.0, 448.0, 2.0 ** -6, 2.0 ** -9, -2.0, 0.0]
    assert np.isnan(E.e4m3_decode(np.array([0x7F]))[0])
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    # Every finite code round-trips (signed zeros included).
    assert np.array_equal(E.e4m3_encode(E.e4m3_decode(codes)), codes)
    # Ties go to the even mantissa; saturation at 448; tiny values keep their sign at zero.
    got = E.e4m3_encode(np.array([1.0625, 1.1875, 460.0, 1e6, -1e6, 2.0 ** -10, -2.0 ** -10]))
    assert got.tolist() == [0x38, 0x3A, 0x7E, 0x7E, 0xFE, 0x00, 0x80]
    # Monotone and nearest: decoded value within half a step of the input.
    x = np.linspace(-448, 448, 4001)
    dec = E.e4m3_decode(E.e4m3_encode(x))
    assert np.all(np.diff(dec) >= 0)
    step = np.maximum(np.abs(dec) * 2.0 ** -3, 2.0 ** -9)
    assert np.all(np.abs(dec - x) <= step / 2 + 1e-12)


def test_bf16_encode_pins():
    assert E.bf16_encode(np.array([1.0, -2.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8], np.float32)).tolist() == \
        [0x3F80, 0xC000, 0x3F80, 0x3F82]
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    d = E.bf16_decode(E.bf16_encode(x))
    assert np.all(np.abs(d - x) <= np.abs(x) * 2.0 ** -8)


def _delta_params(w0_centre: float, latent: int = 4):
    """Encoder 2 -> 8 -> 16 -> 32 -> 64 whose convolutions copy channel co % Ci at the centre tap
    (the first one scaled by w0_centre), zero biases, on a 16^3 input (flat = 64), and a head
    that picks the first `latent` flattened values."""
    chans = (2, 8, 16, 32, 64)
    P = {}
    for i in range(4):
        ci, co = chans[i], chans[i + 1]
        w = torch.zeros(co, ci, 3, 3, 3, dtype=torch.float64)
        for c in range(co):
            w[c, c % ci, 1, 1, 1] = w0_centre if i == 0 else 1.0
        P[f"enc{i}.w"], P[f"enc{i}.b"] = w, torch.zeros(co, dtype=torch.float64)
    P["enc_fc.w"] = torch.eye(latent, 64, dtype=torch.float64)
    P["enc_fc.b"] = torch.zeros(latent, dtype=torch.float64)
    return P


def test_bf16_activation_rounding_and_forward_pins():
    """round_bf16 on hand values (float32 first, then bfloat16 with ties to even), and
    encode_bf16_activations against encode on networks whose activations are copies."""
    v = torch.tensor([0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20,
                      -(1 + 2 ** -8 + 2 ** -20), 1 + 2 ** -8 + 2 ** -30, 3.0], dtype=torch.float64)
    assert E.round_bf16(v).tolist() == [0.0, 1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7,
                                        -(1 + 2 ** -7), 1.0, 3.0]
    # Copies of values k/8 (exact in bfloat16): the rounding changes nothing.
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.integers(0, 9, (2, 2, 16, 16, 16)) / 8.0)
    P = _delta_params(1.0)
    z = E.encode_bf16_activations(P, x)
    assert torch.equal(z, E.encode(P, x))
    assert z[:, 0].tolist() == x[:, 0, 0, 0, 0].tolist() and z[:, 1].tolist() == x[:, 1, 0, 0, 0].tolist()
    # A first layer that scales by 1 + 2^-8 + 2^-20: its output is stored rounded to
    # 1 + 2^-7 (times the input), which the later copies carry to the latent.
    x1 = torch.ones(1, 2, 16, 16, 16, dtype=torch.float64)
    P = _delta_params(1 + 2 ** -8 + 2 ** -20)
    assert E.encode_bf16_activations(P, x1)[0, 0].item() == 1 + 2 ** -7
    assert E.encode(P, x1)[0, 0].item() == 1 + 2 ** -8 + 2 ** -20


def test_hash_oracle_pins():
    """Thresholds, codes, Hamming distances and the Bi-half layer against hand values and
    the identities that tie them to the paper's L2 ranking of +-1 codes."""
    # Lower median: rank (n - 1) // 2.
    X = np.array([[3, 4], [1, 1], [2, 3], [5, 2], [4, 5]], np.float32)
    assert E.hash_thresholds(X).tolist() == [3.0, 3.0]
    assert E.hash_thresholds(X[:4]).tolist() == [2.0, 2.0]
    # Bits: x > t, LSB first; a ramp around 0 sets the upper 16 bits.
    ramp = (np.arange(32, dtype=np.float32) - 15.5)[None, :]
    assert E.binarize(ramp, np.zeros(32, np.float32)).tolist() == [[0xFFFF0000]]
    # Distinct values: every coordinate splits the rows in two halves.
    rng = np.random.default_rng(0)
    for n in (8, 9):
        Y = rng.standard_normal((n, 64)).astype(np.float32)
        c = E.binarize(Y, E.hash_thresholds(Y))
        bits = np.unpackbits(c.view(np.uint8), axis=1, bitorder="little")
        assert np.all(bits.sum(axis=0) == n // 2)
        # The Bi-half layer over the same rows gives the same split (+1 <-> bit 1).
        assert np.array_equal(E.bihalf_forward(Y) > 0, bits.astype(bool))
    # Hamming: 0 to itself, dim to the complement; 4 x Hamming = |b_q - b_x|^2 of the
    # +-1 vectors, so Hamming ranks like the paper's L2 on binary codes.
    Q = E.binarize(rng.standard_normal((5, 96)).astype(np.float32), np.zeros(96, np.float32))
    Xc = E.binarize(rng.standard_normal((7, 96)).astype(np.float32), np.zeros(96, np.float32))
    assert np.all(np.diag(E.hamming(Q, Q)) == 0)
    assert np.all(np.diag(E.hamming(Q, (~Q.view(np.uint32)).view("<u4"))) == 96)
    pm = lambda c: np.unpackbits(c.view(np.uint8), axis=1, bitorder="little").astype(np.float64) * 2 - 1
    l2 = ((pm(Q)[:, None, :] - pm(Xc)[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(4 * E.hamming(Q, Xc).astype(np.float64), l2)
    # Bi-half ties: equal values go to the lower row first; odd B gives floor(B/2) ones.
    T = np.array([[1.0], [1.0], [1.0], [0.0], [1.0]], np.float32)
    assert E.bihalf_forward(T)[:, 0].tolist() == [1, 1, -1, -1, -1]
    # Backward by hand: B = D = 2, gamma = 4 -> dU = G + (U - B).
    U = np.array([[0.5, -1.0], [2.0, 0.0]], np.float64)
    Bc = E.bihalf_forward(U)
    assert Bc.tolist() == [[-1, -1], [1, 1]]
    dU = E.bihalf_backward(U, Bc, np.ones_like(U), 4.0)
    assert dU.tolist() == [[2.5, 1.0], [2.0, 0.0]]


def test_vae_and_l2sum_oracle_pins():
    """KL closed forms, the reparameterisation and the summed L2 of two latent sets."""
    B, L = 3, 4
    ml = torch.zeros(B, 2 * L, dtype=torch.float64)
    eps = torch.randn(B, L, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    z, kl = E.vae_head(ml, eps)
    assert float(kl) == 0.0 and torch.equal(z, eps)          # N(0, 1) itself
    ml[0, 0] = 1.0                                             # one mean of 1: KL = 1/2 / B
    ml[1, L + 2] = np.log(4.0)                                 # one variance of 4
    z, kl = E.vae_head(ml, eps)
    want = (0.5 + -0.5 * (1 + np.log(4.0) - 4.0)) / B
    assert abs(float(kl) - want) < 1e-15
    assert float(z[1, 2]) == 2.0 * float(eps[1, 2]) and float(z[0, 0]) == 1.0 + float(eps[0, 0])
    # Summed L2: orthogonal unit vectors are sqrt(2) apart in each set; a set with itself is 0.
    e = np.eye(4)
    d = E.l2sum_direct(e[:1], e[1:2], e[:1], e[:1])
    assert abs(d[0, 0] - np.sqrt(2.0)) < 1e-15
    rng = np.random.default_rng(1)
    A, Bm = rng.standard_normal((3, 8)), rng.standard_normal((5, 8))
    assert np.allclose(E.l2sum_direct(A, Bm, A, Bm), 2 * np.sqrt(E.sqdist_direct(A, Bm)))
    # Triangle inequality holds for the sum of two metrics.
    C = rng.standard_normal((5, 8))
    lhs = E.l2sum_direct(A, C, A, C)
    rhs = E.l2sum_direct(A, Bm, A, Bm)[:, :, None] + E.l2sum_direct(Bm, C, Bm, C)[None, :, :]
    for i in range(3):
        for j in range(5):
            assert lhs[i, j] <= min(rhs[i, m, j] for m in range(5)) + 1e-12
