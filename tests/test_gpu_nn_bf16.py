"""GPU checks of the encoder's BF16 inference forward (bfloat16 channels-last activations,
each layer's FP32 result rounded to the nearest bfloat16) against the float64 oracle.

Layer contract (the same bfloat16 inputs and weights on both sides), per output element:
|got - want| <= one bfloat16 step of the larger of the two + K 2^-24 S, where want is the
oracle's float64 value stored as bfloat16 (oracle.encoder.round_bf16), K = 27 Ci is the number
of products summed and S the same convolution of absolute values (the bound of a K-term FP32
sum); and at most 1 in 500 outputs differ from want at all. The float-output last layer:
|got - want| <= K 2^-24 S against the float64 value. The whole encoder is within 1e-3
(max-norm relative) of oracle.encoder.encode_bf16_activations: an output stored one
bfloat16 step away moves the latent by about that step times the gain of the later layers."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, say
from oracle import encoder as E

pytestmark = pytest.mark.gpu


def _f64(t):
    return t.detach().to("cpu", torch.float64)


def _rel(a, b):
    return float((a - b).abs().max() / max(b.abs().max(), 1e-30))


def _neighbour_check(got, want, sum_bound):
    """got, want: float64 tensors of bfloat16 values; sum_bound: per element K 2^-24 S.
    Asserts |got - want| <= one bfloat16 step of the larger magnitude + sum_bound; returns the
    fraction of elements that differ."""
    diff = got != want
    if diff.any():
        g, w, sb = got[diff], want[diff], sum_bound[diff]
        m = torch.maximum(g.abs(), w.abs())
        ulp = torch.exp2(torch.floor(torch.log2(m)) - 7)
        ok = (g - w).abs() <= ulp + sb
        assert bool(ok.all()), float(((g - w).abs() / (ulp + sb)).max())
    return float(diff.double().mean())


def _bf16_input(shape, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.relu(torch.randn(shape, generator=g))
    return x.to(torch.bfloat16)


@pytest.mark.parametrize("ci,co,dims,B", [
    (8, 16, (32, 32, 32), 2), (8, 16, (16, 8, 64), 1),      # the workload's layer 2; two x tiles
    (8, 16, (32, 32, 32), 131), (8, 16, (32, 32, 32), 260), # two / four tiles per block
    (16, 32, (16, 16, 16), 2), (16, 32, (8, 16, 32), 1),    # layer 3
    (32, 64, (8, 8, 8), 3), (32, 64, (16, 8, 8), 1),        # layer 4
])
def test_conv_bf16_layer_matches_oracle(ci, co, dims, B):
    need_gpu()
    from paper_2205_04550_amd import nn
    D, H, W = dims
    x = _bf16_input((B, D, H, W, ci), ci + D)                # channels-last
    g = torch.Generator().manual_seed(co)
    w = (torch.randn(co, ci, 3, 3, 3, generator=g) * (2.0 / (27 * ci)) ** 0.5).to(torch.bfloat16)
    bias = torch.randn(co, generator=g) * 0.1
    wtm = nn.conv_weights_tapmajor(w.cuda())
    assert torch.equal(wtm[:, :27].cpu(), w.reshape(co, ci, 27).permute(0, 2, 1))
    assert not wtm[:, 27].any()
    x64 = _f64(x).permute(0, 4, 1, 2, 3).contiguous()        # NCDHW for the oracle
    # Bound of a K-term FP32 sum: K 2^-24 times the sum of the terms' magnitudes.
    sb = 27 * ci * 2.0 ** -24 * E.conv(x64.abs(), _f64(w).abs(), bias.double().abs(), False)
    for relu in (True, False):
        say(f"conv_bf16 {ci}->{co} {dims} B={B} relu={relu}")
        y = nn.conv3d_bf16(x.cuda(), wtm, bias.cuda(), relu)
        yr = E.conv(x64, _f64(w), bias.double(), relu)
        frac = _neighbour_check(_f64(y).permute(0, 4, 1, 2, 3), E.round_bf16(yr), sb)
        say(f"  outputs one step away: {frac:.2e}")
        assert frac <= 2e-3
        yf = nn.conv3d_bf16(x.cuda(), wtm, bias.cuda(), relu, out_f32=True)
        assert yf.shape == yr.shape
        assert bool(((_f64(yf) - yr).abs() <= sb).all())


def test_conv_bf16_rejects_unsupported_shapes():
    need_gpu()
    from paper_2205_04550_amd import nn
    wtm = nn.conv_weights_tapmajor(torch.zeros(16, 8, 3, 3, 3, dtype=torch.bfloat16, device="cuda"))
    with pytest.raises(RuntimeError):                        # W / 2 not a multiple of 16
        nn.conv3d_bf16(torch.zeros(1, 8, 8, 16, 8, dtype=torch.bfloat16, device="cuda"), wtm, None)
    wtm2 = nn.conv_weights_tapmajor(torch.zeros(24, 8, 3, 3, 3, dtype=torch.bfloat16, device="cuda"))
    with pytest.raises(RuntimeError):                        # (Ci, Co) not a built pair
        nn.conv3d_bf16(torch.zeros(1, 8, 8, 32, 8, dtype=torch.bfloat16, device="cuda"), wtm2, None)


def test_first_layer_bf16_is_the_float_layer_rounded():
    """The BF16 first layer stores exactly the float first layer's values rounded to bfloat16
    (same FP32 arithmetic), channels-last; from packed masks it is the same bit for bit."""
    need_gpu()
    from paper_2205_04550_amd import TumorDB, nn
    import synth
    nz = ny = nx = 128
    B = 2
    rng = np.random.default_rng(11)
    lab = rng.integers(0, 4, size=(B, nz, ny, nx), dtype=np.uint8)
    lab[:, :40] = 0
    lab_d = torch.from_numpy(lab).cuda()
    db = TumorDB(nx, ny, nz, 1, synth.T_LO, synth.T_HI)
    db.append(torch.zeros((1, nz, ny, nx), dtype=torch.float32, device="cuda"))
    ws = db.rerank_workspace(B)
    db.rerank_pack(lab_d, ws)
    planes = db.packed_queries(ws, B).clone()
    counts = db.rerank_pack_pool(lab_d, db.rerank_workspace(B))
    g = torch.Generator().manual_seed(4)
    for mask in (None, 0, 1):
        ci = 2 if mask is None else 1
        wc = (torch.randn(8, ci, 3, 3, 3, generator=g) * 0.3).to(torch.bfloat16).cuda()
        b = torch.randn(8, generator=g).cuda()
        for relu in (True, False):
            yf = nn.pool_conv_labels(lab_d, wc, b, relu, mask)
            yb = nn.pool_conv_labels_bf16(lab_d, wc, b, relu, mask)
            assert torch.equal(yb, yf.permute(0, 2, 3, 4, 1).to(torch.bfloat16)), (mask, relu)
            yp = nn.pool_conv_planes_bf16(planes, (nx, ny, nz), wc, b, relu, mask)
            assert torch.equal(yp.view(torch.int16), yb.view(torch.int16)), (mask, relu)
            yc = nn.pool_conv_counts_bf16(counts, wc, b, relu, mask)
            assert torch.equal(yc.view(torch.int16), yb.view(torch.int16)), (mask, relu)


def test_encode_bf16_matches_oracle():
    """The BF16 forward of a whole encoder, after training steps, against
    oracle.encoder.encode_bf16_activations (weights: the model's bfloat16 working copies;
    biases float), and the planes path equal to the labels path bit for bit."""
    need_gpu()
    from paper_2205_04550_amd import TumorDB, nn
    import synth
    gen = synth.FULL
    labels, _ = synth.make_queries(gen, synth.FULL_N, 3, synth.HELDOUT_SEED,
                                   held_out_seed=synth.HELDOUT_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    model = nn.AutoEncoder(grid=64, latent=512, seed=7)
    zb0 = model.encode_labels_bf16(lab_d)                    # the BF16 weight copies made once
    # A few training steps change the working weights in place; the forward must follow.
    opt = nn.Adam(model, lr=1e-2)
    x = nn.meanpool_labels(lab_d)
    for _ in range(3):
        nn.train_step(model, opt, x)
    zb = model.encode_labels_bf16(lab_d)
    assert not torch.equal(zb, zb0)
    P = {}
    for i in range(4):
        P[f"enc{i}.w"] = _f64(model.work[f"enc{i}.w"])
        P[f"enc{i}.b"] = _f64(model.params[f"enc{i}.b"])
    P["enc_fc.w"] = _f64(model.work["enc_fc.w"])
    P["enc_fc.b"] = _f64(model.params["enc_fc.b"])
    x = torch.from_numpy(E.meanpool(labels))
    zr = E.encode_bf16_activations(P, x)
    err = _rel(_f64(zb), zr)
    say(f"BF16 encoder vs oracle: {err:.2e}; vs the float forward: "
        f"{_rel(_f64(zb), _f64(model.encode_labels(lab_d))):.2e}")
    assert err < 1e-3
    nz, ny, nx = labels.shape[1:]
    db = TumorDB(nx, ny, nz, 1, synth.T_LO, synth.T_HI)
    db.append(torch.zeros((1, nz, ny, nx), dtype=torch.float32, device="cuda"))
    ws = db.rerank_workspace(3)
    db.rerank_pack(lab_d, ws)
    zp = model.encode_planes_bf16(db.packed_queries(ws, 3), (nx, ny, nz))
    assert torch.equal(zp, zb)
    zc = model.encode_counts_bf16(db.rerank_pack_pool(lab_d, db.rerank_workspace(3)))
    assert torch.equal(zc, zb)


@pytest.mark.parametrize("dims", [(128, 20, 12), (256, 36, 28)])
def test_first_layer_from_counts_on_ragged_grids(dims):
    """The first layer from pooled counts equals the labels path bit for bit where tiles are
    cut by the grid (output y and z not multiples of the 4 x 2 tile), where a sample has two
    tile columns (the halo count taken from the neighbouring column) and where a block has
    fewer tiles than the launch gives it."""
    need_gpu()
    from paper_2205_04550_amd import TumorDB, nn
    import synth
    nx, ny, nz = dims
    B = 3
    rng = np.random.default_rng(nx + ny)
    lab = rng.integers(0, 4, size=(B, nz, ny, nx), dtype=np.uint8)
    lab[1, :, : ny // 2] = 0
    lab_d = torch.from_numpy(lab).cuda()
    db = TumorDB(nx, ny, nz, 1, synth.T_LO, synth.T_HI)
    db.append(torch.zeros((1, nz, ny, nx), dtype=torch.float32, device="cuda"))
    counts = db.rerank_pack_pool(lab_d, db.rerank_workspace(B))
    g = torch.Generator().manual_seed(9)
    for mask in (None, 0, 1):
        ci = 2 if mask is None else 1
        wc = (torch.randn(8, ci, 3, 3, 3, generator=g) * 0.3).to(torch.bfloat16).cuda()
        b = torch.randn(8, generator=g).cuda()
        for relu in (True, False):
            yb = nn.pool_conv_labels_bf16(lab_d, wc, b, relu, mask)
            yc = nn.pool_conv_counts_bf16(counts, wc, b, relu, mask)
            assert torch.equal(yc.view(torch.int16), yb.view(torch.int16)), (mask, relu)
            yf = nn.pool_conv_labels(lab_d, wc, b, relu, mask)
            assert torch.equal(yb, yf.permute(0, 2, 3, 4, 1).to(torch.bfloat16)), (mask, relu)


@pytest.mark.parametrize("dims", [(96, 10, 6), (64, 64, 64), (128, 128, 128)])
def test_pack_pool_counts_and_packed_queries(dims):
    """db_rerank_pack_pool: the pooled counts are 8x the oracle's 2x2x2 means of both masks
    (exactly), and the packed masks, counts, boxes and moments it leaves in the workspace are
    db_rerank_pack's: the same bits, and the same rerank results bit for bit. Grids with a
    word count per row of 3, lane units that fill some blocks partly and others not at all,
    an empty query, a one-voxel query and an all-set query."""
    need_gpu()
    from paper_2205_04550_amd import TumorDB
    import synth
    nx, ny, nz = dims
    n, nq = 40, 6
    rng = np.random.default_rng(nx + ny + nz)
    lab = rng.integers(0, 4, size=(nq, nz, ny, nx), dtype=np.uint8)
    lab[1] = 0
    lab[2] = 0
    lab[2, nz - 1, ny - 1, nx - 1] = 3
    lab[3] = 3
    lab[4, : nz // 2] = 0
    lab_d = torch.from_numpy(lab).cuda()
    db = TumorDB(nx, ny, nz, n, synth.T_LO, synth.T_HI)
    db.append(torch.from_numpy(rng.random((n, nz, ny, nx), dtype=np.float32)).cuda())
    ws_a, ws_b = db.rerank_workspace(nq), db.rerank_workspace(nq)
    ws_b.fill_(0xA5)                              # the pooled call must write all it reads
    db.rerank_pack(lab_d, ws_a)
    counts = db.rerank_pack_pool(lab_d, ws_b)
    db.sync()
    mp = E.meanpool(lab)                           # float64 [nq][2][nz/2][ny/2][nx/2]
    c = counts.cpu().numpy()
    assert np.array_equal((c & 15).astype(np.float64), 8 * mp[:, 0])
    assert np.array_equal((c >> 4).astype(np.float64), 8 * mp[:, 1])
    assert torch.equal(db.packed_queries(ws_a, nq), db.packed_queries(ws_b, nq))
    cand = torch.from_numpy(np.stack([rng.choice(n, 12, replace=False) for _ in range(nq)])
                            .astype(np.int32)).cuda()
    want = db.rerank_packed(ws_a, cand, 5)
    got = db.rerank_packed(ws_b, cand, 5)
    db.sync()
    for a, w in zip(got, want):
        assert torch.equal(a, w)


def test_pack_pool_rejects_odd_grids_and_bad_pointers():
    need_gpu()
    from paper_2205_04550_amd import TumorDB
    from paper_2205_04550_amd.binding import DbError
    import synth
    db = TumorDB(32, 4, 3, 1, synth.T_LO, synth.T_HI)
    db.append(torch.zeros((1, 3, 4, 32), dtype=torch.float32, device="cuda"))
    lab = torch.zeros((2, 3, 4, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(DbError, match="ny and nz must be even"):
        db.rerank_pack_pool(lab, db.rerank_workspace(2),
                            torch.empty((2, 1, 2, 16), dtype=torch.uint8, device="cuda"))
    db2 = TumorDB(32, 4, 4, 1, synth.T_LO, synth.T_HI)
    db2.append(torch.zeros((1, 4, 4, 32), dtype=torch.float32, device="cuda"))
    lab2 = torch.zeros((2, 4, 4, 32), dtype=torch.uint8, device="cuda")
    buf = torch.empty(2 * 2 * 2 * 16 + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(DbError, match="8-byte aligned"):
        db2.rerank_pack_pool(lab2, db2.rerank_workspace(2), buf[1:].view(2, 2, 2, 16))


@pytest.mark.parametrize("dims,B", [
    ((128, 128, 128), 3),     # the workload's grid; chunks of 4 output slices per block
    ((256, 64, 32), 2),       # two x tiles: the first layer's column x = 2 X0 - 1 computed
    ((128, 32, 48), 1),       # one y tile, three output slices in one chunk
    ((128, 96, 16), 700),     # every slice per block, three y tiles, units % 8 != 0
    ((128, 96, 16), 704),     # the same with the XCD-contiguous unit order
])
def test_first_two_layers_in_one_kernel(dims, B):
    """nn_counts_conv12_bf16 equals the first layer from counts followed by the second BF16
    convolution (two kernels, the activations through memory) bit for bit, for both masks and
    each one alone, with and without biases; counts in 0..8 per mask, a zero region (ReLU of
    the bias alone) and a full region."""
    need_gpu()
    from paper_2205_04550_amd import nn
    nx, ny, nz = dims
    rng = np.random.default_rng(nx + ny + nz + B)
    f = rng.integers(0, 9, size=(B, nz // 2, ny // 2, nx // 2), dtype=np.uint8)
    t = np.minimum(f, rng.integers(0, 9, size=f.shape, dtype=np.uint8))
    f[0, :, : ny // 8] = 0
    t[0, :, : ny // 8] = 0
    f[-1, : nz // 4, :, : nx // 8] = 8
    counts = torch.from_numpy(f | (t << 4)).cuda()
    g = torch.Generator().manual_seed(B)
    for mask, bias in ((None, True), (None, False), (0, True), (1, True)):
        ci = 2 if mask is None else 1
        w1 = (torch.randn(8, ci, 3, 3, 3, generator=g) * 0.3).to(torch.bfloat16).cuda()
        w2 = (torch.randn(16, 8, 3, 3, 3, generator=g) * 0.2).to(torch.bfloat16).cuda()
        b1 = torch.randn(8, generator=g).cuda() * 0.1 if bias else None
        b2 = torch.randn(16, generator=g).cuda() * 0.1 if bias else None
        w2tm = nn.conv_weights_tapmajor(w2)
        want = nn.conv3d_bf16(nn.pool_conv_counts_bf16(counts, w1, b1, True, mask), w2tm, b2, True)
        got = nn.counts_conv12_bf16(counts, w1, b1, w2tm, b2, mask)
        assert got.shape == want.shape
        assert torch.equal(got.view(torch.int16), want.view(torch.int16)), (mask, bias)
        assert float((want != 0).double().mean()) > 0.05


def test_first_two_layers_reject_bad_grids():
    need_gpu()
    from paper_2205_04550_amd import nn
    w1 = torch.zeros(8, 2, 3, 3, 3, dtype=torch.bfloat16, device="cuda")
    w2tm = torch.zeros(16, 28, 8, dtype=torch.bfloat16, device="cuda")
    for pz, py, px in ((8, 16, 32), (8, 8, 64), (4, 16, 64)):   # nx, ny or nz not covered
        c = torch.zeros(1, pz, py, px, dtype=torch.uint8, device="cuda")
        with pytest.raises(RuntimeError):
            nn.counts_conv12_bf16(c, w1, None, w2tm, None)


@pytest.mark.parametrize("B", [1, 3, 300])
def test_third_and_fourth_layers_in_one_kernel(B):
    """nn_conv34_bf16 equals the third and fourth BF16 convolutions as two kernels bit for
    bit, with and without biases, on inputs with zero regions (ReLU of the bias alone)."""
    need_gpu()
    from paper_2205_04550_amd import nn
    x = _bf16_input((B, 16, 16, 16, 16), B)
    x[0, :4] = 0
    x = x.cuda()
    g = torch.Generator().manual_seed(B + 1)
    for bias in (True, False):
        w3 = (torch.randn(32, 16, 3, 3, 3, generator=g) * 0.1).to(torch.bfloat16).cuda()
        w4 = (torch.randn(64, 32, 3, 3, 3, generator=g) * 0.1).to(torch.bfloat16).cuda()
        b3 = torch.randn(32, generator=g).cuda() * 0.1 if bias else None
        b4 = torch.randn(64, generator=g).cuda() * 0.1 if bias else None
        t3, t4 = nn.conv_weights_tapmajor(w3), nn.conv_weights_tapmajor(w4)
        want = nn.conv3d_bf16(nn.conv3d_bf16(x, t3, b3, True), t4, b4, True, out_f32=True)
        got = nn.conv34_bf16(x, t3, b3, t4, b4)
        assert torch.equal(got.view(torch.int32), want.view(torch.int32)), bias
        assert float((want != 0).double().mean()) > 0.05
