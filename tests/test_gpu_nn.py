"""GPU checks of the encoder kernels: layer parity with the float64 CPU oracle, gradients
against the oracle's autograd and against finite differences, mean-pooling, Adam and BF16."""
import math

import numpy as np
import pytest
import torch

import synth
from gpu_util import build_db_from_host, need_gpu, say
from oracle import encoder as E

pytestmark = pytest.mark.gpu


def _cpu64(t):
    return t.detach().to("cpu", torch.float64)


def _rel(a, b):
    return float((a - b).abs().max() / max(b.abs().max(), 1e-30))


def _within_sum_bound(y, yr, S, K):
    """Per element: |y - yr| <= (K + 2) 2^-24 S, the error of a K-term FP32 sum of rounded
    products (S: the same sum of the terms' magnitudes) plus the rounding of the inputs."""
    err = (_cpu64(y) - yr).abs()
    bound = (K + 2) * 2.0 ** -24 * S
    return bool((err <= bound).all()), float((err / bound.clamp_min(1e-300)).max())


def test_meanpool_db_and_labels_exact():
    need_gpu()
    from paper_2205_04550_amd import nn
    gen = synth.GenConfig(64, 32, 16, 2.0, 10.0, 0.5, 3.0, 12)
    n = 9
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    import oracle
    labs = np.stack([oracle.threshold(c, synth.T_LO, synth.T_HI) for c in conc])
    idx = torch.tensor([3, 0, 8, 3], dtype=torch.int32, device="cuda")
    for dt in (torch.float32, torch.float64):
        got = nn.meanpool_db(db, idx, dt).cpu().numpy()
        want = E.meanpool(labs[[3, 0, 8, 3]])
        assert np.array_equal(got.astype(np.float64), want)
        got2 = nn.meanpool_labels(torch.from_numpy(labs).cuda(), dt).cpu().numpy()
        assert np.array_equal(got2.astype(np.float64), E.meanpool(labs))


def _magnitudes(f, x, w, b, gy):
    """For a layer f(x, w, b) linear in x, in w and in b: the sums of the magnitudes of the
    terms of every output and of every gradient entry for the upstream gradient gy (the same
    operations on absolute values; the gradients through autograd of the oracle)."""
    xa, wa, ba, ga = x.detach().abs(), w.detach().abs(), b.detach().abs(), gy.abs()
    Sy = f(xa, wa, ba)
    xg = xa.clone().requires_grad_(True)
    (Sgx,) = torch.autograd.grad((f(xg, wa, None) * ga).sum(), xg)
    wg = wa.clone().requires_grad_(True)
    (Sgw,) = torch.autograd.grad((f(xa, wg, None) * ga).sum(), wg)
    bg = ba.clone().requires_grad_(True)
    (Sgb,) = torch.autograd.grad((f(xa, wa, bg) * ga).sum(), bg)
    return Sy, Sgx, Sgw, Sgb


def _check_layer(f, x64, w_ref, b64, relu, y, grads, K, u):
    """y and the GPU gradients (x, w, b) against the oracle, per element:
    |got - want| <= (K + 2) u S, S from _magnitudes, u the unit roundoff of the dtype."""
    xr = x64.clone().requires_grad_(True)
    wr = w_ref.clone().requires_grad_(True)
    br = b64.clone().requires_grad_(True)
    pre = f(xr, wr, br)
    yr = torch.relu(pre) if relu else pre
    gy = grads[0]
    gy_eff = gy * (pre > 0) if relu else gy                 # the upstream gradient through ReLU
    (yr * gy).sum().backward()
    S = _magnitudes(f, x64, w_ref, b64, gy_eff)
    for name, got, want, Sk in (("y", y, yr.detach(), S[0]), ("dx", grads[1], xr.grad, S[1]),
                                ("dw", grads[2], wr.grad, S[2]), ("db", grads[3], br.grad, S[3])):
        err = (_cpu64(got) - want).abs()
        bound = (K + 2) * u * Sk
        assert bool((err <= bound).all()), (name, float((err / bound.clamp_min(1e-300)).max()))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_layers_match_oracle_forward_and_backward(dtype):
    """Convolution, transposed convolution and linear layer, forward and all three gradients,
    against the float64 oracle (its autograd for the gradients), every element within the
    bound of its own sum (K terms, unit roundoff u of the dtype)."""
    need_gpu()
    from paper_2205_04550_amd import nn
    torch.manual_seed(0)
    B, Ci, Co, D, H, W = 3, 5, 7, 10, 8, 6
    x64 = torch.randn(B, Ci, D, H, W, dtype=torch.float64)
    w64 = torch.randn(Co, Ci, 3, 3, 3, dtype=torch.float64) * 0.2
    b64 = torch.randn(Co, dtype=torch.float64)
    if dtype == torch.float32:
        wc = w64.to(torch.bfloat16)                  # the kernels' BF16 working weights
        w_ref = wc.to(torch.float64)
        u = 2.0 ** -24
    else:
        wc = None
        w_ref = w64
        u = 2.0 ** -53
    # Terms per sum: at most 27 max(Ci, Co) for outputs and input gradients, B x (output
    # voxels) for weight and bias gradients.
    K = 27 * max(Ci, Co) + B * D * H * W
    xs = x64.to("cuda", dtype).requires_grad_(True)
    ws = w64.to("cuda", dtype).requires_grad_(True)
    bs = b64.to("cuda", dtype).requires_grad_(True)
    wcs = wc.cuda() if wc is not None else ws.detach()
    conv = lambda x, w, b: E.conv(x, w, b, False)
    for relu in (False, True):
        say(f"conv {dtype} relu={relu}")
        y = nn.Conv3dS2.apply(xs, ws, bs, wcs, relu)
        gy = torch.randn(y.shape, dtype=torch.float64)
        g = torch.autograd.grad(y, (xs, ws, bs), gy.to("cuda", dtype))
        _check_layer(conv, x64, w_ref, b64, relu, y, (gy,) + g, K, u)
    # transposed conv: weight [Cin][Cout] with Cin = Co here (maps Co -> Ci channels)
    xt64 = torch.randn(B, Co, D // 2, H // 2, W // 2, dtype=torch.float64)
    bt64 = torch.randn(Ci, dtype=torch.float64)
    xts = xt64.to("cuda", dtype).requires_grad_(True)
    bts = bt64.to("cuda", dtype).requires_grad_(True)
    convt = lambda x, w, b: E.conv_t(x, w, b, False)
    for relu in (False, True):
        say(f"convT {dtype} relu={relu}")
        y = nn.ConvT3dS2.apply(xts, ws, bts, wcs, relu)
        assert y.shape == (B, Ci, D, H, W)
        gy = torch.randn(y.shape, dtype=torch.float64)
        g = torch.autograd.grad(y, (xts, ws, bts), gy.to("cuda", dtype))
        _check_layer(convt, xt64, w_ref, bt64, relu, y, (gy,) + g, K, u)
    # linear
    In, Out = 37, 19
    xl64 = torch.randn(B, In, dtype=torch.float64)
    wl64 = torch.randn(Out, In, dtype=torch.float64) * 0.3
    bl64 = torch.randn(Out, dtype=torch.float64)
    wlc = wl64.to(torch.bfloat16).cuda() if dtype == torch.float32 else None
    wl_ref = wl64.to(torch.bfloat16).to(torch.float64) if dtype == torch.float32 else wl64
    xls = xl64.to("cuda", dtype).requires_grad_(True)
    wls = wl64.to("cuda", dtype).requires_grad_(True)
    bls = bl64.to("cuda", dtype).requires_grad_(True)
    lin = lambda x, w, b: torch.nn.functional.linear(x, w, b)
    for relu in (False, True):
        say(f"linear {dtype} relu={relu}")
        y = nn.Linear.apply(xls, wls, bls, wlc if wlc is not None else wls.detach(), relu)
        gy = torch.randn(y.shape, dtype=torch.float64)
        g = torch.autograd.grad(y, (xls, wls, bls), gy.to("cuda", dtype))
        _check_layer(lin, xl64, wl_ref, bl64, relu, y, (gy,) + g, max(In, Out, B) + 2, u)


def test_gradcheck_float64_functions():
    need_gpu()
    from paper_2205_04550_amd import nn
    torch.manual_seed(1)
    d = dict(dtype=torch.float64, device="cuda")
    x = torch.randn(2, 2, 4, 4, 4, **d, requires_grad=True)
    w = torch.randn(3, 2, 3, 3, 3, **d, requires_grad=True)
    b = torch.randn(3, **d, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x, w, b: nn.Conv3dS2.apply(x, w, b, w, False),
                                    (x, w, b), eps=1e-6, atol=1e-8, rtol=1e-6)
    xt = torch.randn(2, 3, 2, 2, 2, **d, requires_grad=True)
    bt = torch.randn(2, **d, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x, w, b: nn.ConvT3dS2.apply(x, w, b, w, False),
                                    (xt, w, bt), eps=1e-6, atol=1e-8, rtol=1e-6)
    xl = torch.randn(3, 6, **d, requires_grad=True)
    wl = torch.randn(4, 6, **d, requires_grad=True)
    bl = torch.randn(4, **d, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x, w, b: nn.Linear.apply(x, w, b, w, False),
                                    (xl, wl, bl), eps=1e-6, atol=1e-8, rtol=1e-6)
    a = torch.randn(5, 3, **d, requires_grad=True)
    t = torch.randn(5, 3, **d)
    assert torch.autograd.gradcheck(lambda a: nn.MSE.apply(a, t), (a,), eps=1e-6, atol=1e-8)


def test_autoencoder_finite_differences_16cube():
    """Whole autoencoder in float64 on a 16^3 instance (16 -> 8 -> 4 -> 2 -> 1, 64 channels,
    latent 512, mirrored decoder), batch 2: analytic gradients of the MSE loss against
    central differences (h = 1e-6) for every bias and 200 random entries of every weight
    and of the input."""
    need_gpu()
    from paper_2205_04550_amd import nn
    model = nn.AutoEncoder(grid=16, latent=512, dtype=torch.float64, seed=3)
    torch.manual_seed(4)
    # Random biases: with zero biases, units whose inputs are all zero sit exactly on the
    # ReLU kink, where the derivative is one-sided and central differences see half of it.
    with torch.no_grad():
        for k, p in model.params.items():
            if k.endswith(".b"):
                p.copy_(torch.randn(p.shape, dtype=torch.float64) * 0.1)
    x = torch.rand(2, 2, 16, 16, 16, dtype=torch.float64, device="cuda").requires_grad_(True)
    target = x.detach().clone()   # the reconstruction target stays fixed when x is perturbed

    def loss_of(inp):
        return nn.MSE.apply(model.forward(inp), target)

    loss = loss_of(x)
    loss.backward()
    # forward agrees with the oracle
    params_cpu = {k: _cpu64(p) for k, p in model.params.items()}
    ref = E.mse(E.decode(params_cpu, E.encode(params_cpu, _cpu64(x)), 64, 1), _cpu64(x))
    assert abs(float(loss.detach()) - float(ref)) <= 1e-12 * abs(float(ref))
    h = 1e-6
    l0 = float(loss.detach())
    rng = np.random.default_rng(5)
    tensors = [(k, p) for k, p in model.params.items()] + [("input", x)]
    checked = skipped = 0
    for name, p in tensors:
        g = p.grad.detach().cpu().numpy().ravel()
        flat = p.data.view(-1)
        if name.endswith(".b"):
            coords = range(flat.numel())
        else:
            coords = rng.choice(flat.numel(), size=min(200, flat.numel()), replace=False)
        gmax = float(np.abs(g).max())
        for c in coords:
            c = int(c)
            old = float(flat[c])
            flat[c] = old + h
            lp = float(loss_of(x.detach()))
            flat[c] = old - h
            lm = float(loss_of(x.detach()))
            flat[c] = old
            fd = (lp - lm) / (2 * h)
            # A ReLU switching inside [-h, h] makes the one-sided slopes disagree: skip it.
            if abs((lp - l0) / h - (l0 - lm) / h) > 1e-3 * abs(fd) + 1e-6:
                skipped += 1
                continue
            assert abs(fd - g[c]) <= 1e-5 * abs(g[c]) + 1e-7 * gmax + 1e-9, (name, c, fd, g[c])
            checked += 1
    assert skipped <= 0.01 * (checked + skipped)
    say(f"finite differences: {checked} coordinates agree, {skipped} skipped at ReLU kinks")


def test_bf16_rounding_and_adam_step():
    need_gpu()
    from paper_2205_04550_amd import nn
    from paper_2205_04550_amd.binding import LIB, _check
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)).astype(np.float32)
    x[:4] = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0], np.float32)  # ties
    u = x.view(np.uint32).astype(np.uint64)
    want = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)    # round to nearest even
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty(x.size, dtype=torch.bfloat16, device="cuda")
    _check(LIB.nn_to_bf16(x.size, xd.data_ptr(), yd.data_ptr(), torch.cuda.current_stream().cuda_stream))
    got = yd.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, want)
    # one Adam step against the textbook formula in float32 (numpy)
    w = rng.standard_normal(513).astype(np.float32)
    g = rng.standard_normal(513).astype(np.float32)
    m = rng.standard_normal(513).astype(np.float32) * 0.1
    v = np.abs(rng.standard_normal(513).astype(np.float32)) * 0.1
    lr, b1, b2, eps, t = 1e-3, 0.9, 0.999, 1e-8, 3
    W, M, Vv, G = (torch.from_numpy(a.copy()).cuda() for a in (w, m, v, g))
    wb = torch.empty(513, dtype=torch.bfloat16, device="cuda")
    _check(LIB.nn_adam_step(513, W.data_ptr(), M.data_ptr(), Vv.data_ptr(), G.data_ptr(),
                            wb.data_ptr(), lr, b1, b2, eps, t, torch.cuda.current_stream().cuda_stream))
    m2 = np.float32(b1) * m + np.float32(1 - b1) * g
    v2 = np.float32(b2) * v + np.float32(1 - b2) * g * g
    w2 = w - np.float32(lr) * (m2 / np.float32(1 - b1 ** t)) / (np.sqrt(v2 / np.float32(1 - b2 ** t)) + np.float32(eps))
    assert np.allclose(M.cpu().numpy(), m2, rtol=1e-6, atol=1e-7)
    assert np.allclose(Vv.cpu().numpy(), v2, rtol=1e-6, atol=1e-7)
    assert np.allclose(W.cpu().numpy(), w2, rtol=1e-6, atol=1e-6)
    assert torch.equal(wb, W.to(torch.bfloat16))


def test_training_overfits_one_batch():
    """Forward, backward and Adam together: repeated steps on one batch must drive its
    reconstruction loss well down."""
    need_gpu()
    from paper_2205_04550_amd import nn
    gen = synth.SMALL
    n = 64
    db, _ = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    model = nn.AutoEncoder(grid=32, latent=64, seed=0)
    opt = nn.Adam(model, lr=2e-3)
    idx = torch.arange(0, 64, 8, dtype=torch.int32, device="cuda")
    x = nn.meanpool_db(db, idx)
    losses = [float(nn.train_step(model, opt, x)) for _ in range(150)]
    say(f"loss {losses[0]:.5f} -> {min(losses):.5f} (last {losses[-1]:.5f})")
    assert all(math.isfinite(l) for l in losses)
    assert np.mean(losses[-10:]) < 0.5 * losses[0]


@pytest.mark.parametrize("shape", [(2, 2, 8, 64), (2, 8, 16, 32), (1, 3, 12, 32), (2, 16, 32, 16)])
def test_conv_forward_large_layers(shape):
    """The encoder's large layers (LDS-tiled kernel) against the float64 oracle."""
    need_gpu()
    from paper_2205_04550_amd import nn
    B, Ci, Co, G = shape
    g = torch.Generator().manual_seed(Ci * 100 + Co)
    x64 = torch.rand(B, Ci, G, G, G, generator=g, dtype=torch.float64)
    w64 = torch.randn(Co, Ci, 3, 3, 3, generator=g, dtype=torch.float64) * 0.2
    b64 = torch.randn(Co, generator=g, dtype=torch.float64)
    wc = w64.to(torch.bfloat16)
    for relu in (False, True):
        y = nn.Conv3dS2.apply(x64.to("cuda", torch.float32), w64.cuda().float(), b64.cuda().float(),
                              wc.cuda(), relu)
        yr = E.conv(x64, wc.to(torch.float64), b64, relu)
        S = E.conv(x64.abs(), wc.to(torch.float64).abs(), b64.abs(), False)
        ok, worst = _within_sum_bound(y, yr, S, 27 * Ci)
        assert ok, (shape, relu, worst)


@pytest.mark.parametrize("shape", [(70, 4100, 130), (1024, 4096, 512), (32, 512, 4096), (5, 8, 3)])
def test_linear_forward_matrix_core(shape):
    """Float linear forward on the FP32 matrix cores (K a multiple of 4), several tiles with
    ragged edges in M, N and K, BF16 and float weights, against the float64 oracle product."""
    need_gpu()
    from paper_2205_04550_amd import nn
    B, In, Out = shape
    g = torch.Generator().manual_seed(B + In + Out)
    x64 = torch.randn(B, In, generator=g, dtype=torch.float64)
    w64 = torch.randn(Out, In, generator=g, dtype=torch.float64) * (1.0 / math.sqrt(In))
    b64 = torch.randn(Out, generator=g, dtype=torch.float64)
    for wdt in (torch.bfloat16, torch.float32):
        wc = w64.to(wdt)
        for relu in (False, True):
            say(f"linear mfma {shape} {wdt} relu={relu}")
            y = nn.Linear.apply(x64.to("cuda", torch.float32), w64.cuda().float(),
                                b64.cuda().float(), wc.cuda(), relu)
            yr = x64 @ wc.to(torch.float64).T + b64
            yr = torch.relu(yr) if relu else yr
            S = x64.abs() @ wc.to(torch.float64).abs().T + b64.abs()
            ok, worst = _within_sum_bound(y, yr, S, In)
            assert ok, (shape, wdt, relu, worst)


@pytest.mark.parametrize("shape", [(1024, 4096, 512), (70, 1000, 130), (5, 8, 3)])
def test_linear_split_forward(shape):
    """The head's split-K forward: with one slice the unsplit kernel's bits; with 4, 7 and 8
    slices (some empty when K is small, the last one ragged) within the FP32 sum bound of the
    float64 product and the same bits on a second call."""
    need_gpu()
    from paper_2205_04550_amd import nn
    B, In, Out = shape
    g = torch.Generator().manual_seed(B + In + Out + 1)
    x64 = torch.randn(B, In, generator=g, dtype=torch.float64)
    w64 = torch.randn(Out, In, generator=g, dtype=torch.float64) * (1.0 / math.sqrt(In))
    b64 = torch.randn(Out, generator=g, dtype=torch.float64)
    wc = w64.to(torch.bfloat16)
    x = x64.to("cuda", torch.float32)
    for relu in (False, True):
        want = nn.Linear.apply(x, w64.cuda().float(), b64.cuda().float(), wc.cuda(), relu)
        y1 = nn.linear_split(x, wc.cuda(), b64.cuda().float(), relu, splits=1)
        assert torch.equal(y1, want), (shape, relu)
        yr = x64 @ wc.to(torch.float64).T + b64
        yr = torch.relu(yr) if relu else yr
        S = x64.abs() @ wc.to(torch.float64).abs().T + b64.abs()
        for splits in (4, 7, 8):
            y = nn.linear_split(x, wc.cuda(), b64.cuda().float(), relu, splits=splits)
            ok, worst = _within_sum_bound(y, yr, S, In)
            assert ok, (shape, relu, splits, worst)
            assert torch.equal(y, nn.linear_split(x, wc.cuda(), b64.cuda().float(), relu,
                                                  splits=splits))


@pytest.mark.parametrize("shape", [(3, 4, 20, 14, 10, 40), (2, 32, 64, 8, 8, 8), (2, 20, 16, 18, 12, 20),
                                   (1, 8, 16, 32, 32, 32), (2, 16, 33, 6, 22, 12), (2, 12, 8, 4, 6, 36)])
def test_conv_forward_matrix_core(shape):
    """Float convolution forward on the FP32 matrix cores (Ci, W % 4 == 0): every voxel-box
    shape, one to four 16-channel output tiles with a ragged last tile, several input
    channel chunks, ragged boxes at the volume's edges; BF16 and float weights."""
    need_gpu()
    from paper_2205_04550_amd import nn
    B, Ci, Co, D, H, W = shape
    g = torch.Generator().manual_seed(Ci * 1000 + Co * 10 + D)
    x64 = torch.rand(B, Ci, D, H, W, generator=g, dtype=torch.float64) - 0.3
    w64 = torch.randn(Co, Ci, 3, 3, 3, generator=g, dtype=torch.float64) * 0.2
    b64 = torch.randn(Co, generator=g, dtype=torch.float64)
    for wdt in (torch.bfloat16, torch.float32):
        wc = w64.to(wdt)
        for relu in (False, True):
            say(f"conv mfma {shape} {wdt} relu={relu}")
            y = nn.Conv3dS2.apply(x64.to("cuda", torch.float32), w64.cuda().float(),
                                  b64.cuda().float(), wc.cuda(), relu)
            yr = E.conv(x64, wc.to(torch.float64), b64, relu)
            assert y.shape == yr.shape
            S = E.conv(x64.abs(), wc.to(torch.float64).abs(), b64.abs(), False)
            ok, worst = _within_sum_bound(y, yr, S, 27 * Ci)
            assert ok, (shape, wdt, relu, worst)


@pytest.mark.parametrize("dims", [(12, 20, 256), (8, 8, 128), (128, 128, 128)])
def test_pool_conv_labels_matches_oracle(dims):
    """The first encoder layer read straight from labels (pooling fused, BF16 matrix cores)
    against the float64 oracle conv of the oracle mean-pool: both masks and each mask alone,
    ragged output boxes in z and y, two x tiles (the left halo column of the second)."""
    need_gpu()
    from paper_2205_04550_amd import nn
    nz, ny, nx = dims
    B = 3 if nz < 128 else 2
    rng = np.random.default_rng(nz + ny + nx)
    lab = rng.integers(0, 4, size=(B, nz, ny, nx), dtype=np.uint8)
    lab[:, : nz // 3] = 0                                    # an empty slab
    lab[0, :, :, nx // 2:] &= 1                              # FLAIR without T1Gd
    pooled = E.meanpool(lab)
    g = torch.Generator().manual_seed(nx)
    lab_d = torch.from_numpy(lab).cuda()
    for mask in (None, 0, 1):
        ci = 2 if mask is None else 1
        w64 = torch.randn(8, ci, 3, 3, 3, generator=g, dtype=torch.float64) * 0.3
        b64 = torch.randn(8, generator=g, dtype=torch.float64)
        wc = w64.to(torch.bfloat16)
        x64 = torch.from_numpy(pooled if mask is None else pooled[:, mask:mask + 1].copy())
        for relu in (True, False):
            say(f"pool_conv_labels {dims} mask={mask} relu={relu}")
            y = nn.pool_conv_labels(lab_d, wc.cuda(), b64.cuda().float(), relu, mask)
            yr = E.conv(x64, wc.to(torch.float64), b64, relu)
            assert y.shape == yr.shape
            S = E.conv(x64.abs(), wc.to(torch.float64).abs(), b64.abs(), False)
            ok, worst = _within_sum_bound(y, yr, S, 27 * ci)
            assert ok, (dims, mask, relu, worst)


@pytest.mark.parametrize("dims", [(12, 20, 256), (8, 8, 128), (128, 128, 128)])
def test_pool_conv_planes_equals_pool_conv_labels(dims):
    """The first layer from the queries' packed masks (as db_rerank_pack leaves them) equals
    the first layer from their label bytes bit for bit: both masks and each alone, ragged
    output boxes, two x tiles, samples chosen and reordered by idx."""
    need_gpu()
    from paper_2205_04550_amd import TumorDB, nn
    nz, ny, nx = dims
    B = 3
    rng = np.random.default_rng(nz * ny + nx)
    lab = rng.integers(0, 4, size=(B, nz, ny, nx), dtype=np.uint8)
    lab[:, : nz // 3] = 0
    lab[1, :, :, : nx // 2] &= 2                             # T1Gd without FLAIR
    lab_d = torch.from_numpy(lab).cuda()
    db = TumorDB(nx, ny, nz, 1, synth.T_LO, synth.T_HI)
    db.append(torch.zeros((1, nz, ny, nx), dtype=torch.float32, device="cuda"))
    ws = db.rerank_workspace(B)
    db.rerank_pack(lab_d, ws)
    planes = db.packed_queries(ws, B).clone()
    g = torch.Generator().manual_seed(nz)
    idx = torch.tensor([2, 0], dtype=torch.int32, device="cuda")
    for mask in (None, 0, 1):
        ci = 2 if mask is None else 1
        wc = (torch.randn(8, ci, 3, 3, 3, generator=g) * 0.3).to(torch.bfloat16).cuda()
        b = torch.randn(8, generator=g).cuda()
        for relu in (True, False):
            y1 = nn.pool_conv_labels(lab_d, wc, b, relu, mask)
            y2 = nn.pool_conv_planes(planes, (nx, ny, nz), wc, b, relu, mask)
            assert torch.equal(y1.view(torch.int32), y2.view(torch.int32)), (mask, relu)
        y3 = nn.pool_conv_planes(planes, (nx, ny, nz), wc, b, True, mask, idx)
        assert torch.equal(y3, nn.pool_conv_labels(lab_d[[2, 0]].contiguous(), wc, b, True, mask))


def test_pool_conv_planes_from_the_database():
    """Database entries (their stored bit planes, idx) encode as the labels thresholded from
    the same densities: the fused first layer from planes equals the one from labels."""
    need_gpu()
    from paper_2205_04550_amd import nn
    gen = synth.FULL
    db, conc = build_db_from_host(gen, 4, synth.T_LO, synth.T_HI)
    import oracle
    lab = np.stack([oracle.threshold(c, synth.T_LO, synth.T_HI).reshape(gen.nz, gen.ny, gen.nx)
                    for c in conc])
    g = torch.Generator().manual_seed(2)
    wc = (torch.randn(8, 2, 3, 3, 3, generator=g) * 0.3).to(torch.bfloat16).cuda()
    b = torch.randn(8, generator=g).cuda()
    idx = torch.tensor([3, 1, 1], dtype=torch.int32, device="cuda")
    y_p = nn.pool_conv_planes(db.planes, (gen.nx, gen.ny, gen.nz), wc, b, True, None, idx)
    y_l = nn.pool_conv_labels(torch.from_numpy(lab[[3, 1, 1]]).cuda(), wc, b, True, None)
    assert torch.equal(y_p, y_l)


def test_encode_labels_matches_two_step_encode():
    """AutoEncoder.encode_labels (fused first layer) equals encode(meanpool_labels(.)) up to
    FP32 summation order, for the two-mask encoder and a one-mask encoder."""
    need_gpu()
    from paper_2205_04550_amd import nn
    rng = np.random.default_rng(5)
    lab = torch.from_numpy(rng.integers(0, 4, size=(4, 128, 128, 128), dtype=np.uint8)).cuda()
    for mask, ch in ((None, (2, 8, 16, 32, 64)), (1, (1, 8, 16, 32, 64))):
        model = nn.AutoEncoder(grid=64, channels=ch, latent=512, seed=3)
        with torch.no_grad():
            z1 = model.encode_labels(lab, mask=mask)
            z2 = model.encode(nn.meanpool_labels(lab, mask=mask))
        assert _rel(z1.double().cpu(), z2.double().cpu()) < 1e-4, mask


@pytest.mark.parametrize("shape", [(70, 4100, 132), (32, 4096, 512), (32, 512, 4096), (5, 8, 4)])
def test_linear_input_gradient_matrix_core(shape):
    """Input gradient dY W of the linear layer on the FP32 matrix cores (In, Out % 4 == 0),
    ragged tiles in every dimension, BF16 and float weights, against the float64 product."""
    need_gpu()
    from paper_2205_04550_amd import nn
    B, In, Out = shape
    g = torch.Generator().manual_seed(B * 7 + In + Out)
    x64 = torch.randn(B, In, generator=g, dtype=torch.float64)
    w64 = torch.randn(Out, In, generator=g, dtype=torch.float64) * (1.0 / math.sqrt(Out))
    gy64 = torch.randn(B, Out, generator=g, dtype=torch.float64)
    for wdt in (torch.bfloat16, torch.float32):
        wc = w64.to(wdt)
        say(f"linear dX mfma {shape} {wdt}")
        x = x64.to("cuda", torch.float32).requires_grad_(True)
        y = nn.Linear.apply(x, w64.cuda().float(), None, wc.cuda(), False)
        (gx,) = torch.autograd.grad(y, (x,), gy64.to("cuda", torch.float32))
        ref = gy64 @ wc.to(torch.float64)
        ok, worst = _within_sum_bound(gx, ref, gy64.abs() @ wc.to(torch.float64).abs(), Out)
        assert ok, (shape, wdt, worst)
