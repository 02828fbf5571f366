"""GPU checks of the two-encoder / VAE variant (F4): single-mask mean-pooling, the
summed L2 of two latent sets, the variational head, and finite differences of a small
variational autoencoder in float64."""
import numpy as np
import pytest
import torch

import oracle.encoder as E
import synth
from gpu_util import build_db_from_host, need_gpu, say

pytestmark = pytest.mark.gpu


def _lat(n, dim, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(n, dim, generator=g).to(torch.float32)


def _dequant(L):
    from paper_2205_04550_amd import binding as b
    if L.fmt == b.EMB_BF16:
        return E.bf16_decode(L.codes.view(torch.int16).cpu().numpy())
    return E.e4m3_decode(L.codes.cpu().numpy()) * L.scale.cpu().numpy().astype(np.float64)[:, None]


def test_single_mask_meanpool_exact():
    need_gpu()
    from paper_2205_04550_amd import nn
    gen = synth.SMALL
    db, conc = build_db_from_host(gen, 40, synth.T_LO, synth.T_HI)
    idx = torch.arange(3, 40, 3, dtype=torch.int32, device="cuda")
    both = nn.meanpool_db(db, idx)
    labels, _ = synth.make_queries(gen, 40, 3, synth.QUERY_SEED)
    lab = torch.from_numpy(labels).cuda()
    qboth = nn.meanpool_labels(lab)
    want = E.meanpool(labels)
    for m in (0, 1):
        assert torch.equal(nn.meanpool_db(db, idx, mask=m)[:, 0], both[:, m])
        got = nn.meanpool_labels(lab, mask=m)[:, 0]
        assert torch.equal(got, qboth[:, m])
        assert np.array_equal(got.cpu().numpy().astype(np.float64), want[:, m])


@pytest.mark.parametrize("fmt", [0, 1])
def test_l2sum_within_contract(fmt):
    need_gpu()
    from paper_2205_04550_amd import binding as b
    M, N, dim = 45, 1301, 512
    Q1, Q2 = b.Latents(_lat(M, dim, 1).cuda(), fmt), b.Latents(_lat(M, dim, 2).cuda(), fmt)
    X1 = b.Latents(torch.cat([_lat(M, dim, 1)[:4], _lat(N - 4, dim, 3)]).cuda(), fmt)
    X2 = b.Latents(torch.cat([_lat(M, dim, 2)[:4], _lat(N - 4, dim, 4)]).cuda(), fmt)
    D = b.emb_distances_l2sum(Q1, X1, Q2, X2).cpu().numpy().astype(np.float64)
    q1, x1, q2, x2 = map(_dequant, (Q1, X1, Q2, X2))
    want = E.l2sum_direct(q1, x1, q2, x2)
    # Each squared distance is within rel * (|q|^2 + |x|^2) (the distance contract);
    # |sqrt(a) - sqrt(b)| <= sqrt(|a - b|), plus float rounding of the roots and the sum.
    rel = 1e-5                     # the distance contract, both formats
    bnd = sum(np.sqrt(rel * ((q ** 2).sum(1)[:, None] + (x ** 2).sum(1)[None, :]))
              for q, x in ((q1, x1), (q2, x2)))
    err = np.abs(D - want)
    say(f"fmt {fmt}: max err / bound = {(err / (bnd + 1e-6 * want)).max():.3g}")
    assert np.all(err <= bnd + 1e-6 * want)
    # Self pairs (entries 0..3 are the first queries): both terms near zero.
    assert np.all(np.diag(D[:4, :4]) <= np.diag(bnd[:4, :4]) + 1e-6)
    # Selection on the summed distances is the exact k smallest of D.
    Dd = torch.from_numpy(D.astype(np.float32)).cuda()
    idx, val = b.emb_topk_min(Dd, 50)
    assert np.array_equal(idx.cpu().numpy(), E.topk_by_distance(D.astype(np.float32), 50))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vae_head_matches_oracle(dtype):
    need_gpu()
    from paper_2205_04550_amd import nn
    g = torch.Generator().manual_seed(6)
    B, L = 5, 300
    ml = (torch.randn(B, 2 * L, generator=g, dtype=torch.float64) * 0.7).to(dtype)
    eps = torch.randn(B, L, generator=g, dtype=torch.float64).to(dtype)
    dz = torch.randn(B, L, generator=g, dtype=torch.float64).to(dtype)
    beta = 0.25
    mld = ml.cuda().requires_grad_(True)
    kl = torch.empty((), dtype=dtype, device="cuda")
    z = nn.VaeHead.apply(mld, eps.cuda(), beta, kl)
    z.backward(dz.cuda())
    m64 = ml.to(torch.float64).requires_grad_(True)
    z64, kl64 = E.vae_head(m64, eps.to(torch.float64))
    (z64 * dz.to(torch.float64)).sum().add(beta * kl64).backward()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert float((z.detach().cpu().double() - z64.detach()).abs().max()) <= tol * float(z64.abs().max())
    assert abs(float(kl) - float(kl64)) <= tol * abs(float(kl64))
    gr = mld.grad.cpu().double()
    assert float((gr - m64.grad).abs().max()) <= tol * float(m64.grad.abs().max())


def test_vae_finite_differences_16cube():
    """Single-mask variational autoencoder in float64 on a 16^3 instance, batch 2:
    analytic gradients of MSE + beta * KL (fixed eps) against central differences."""
    need_gpu()
    from paper_2205_04550_amd import nn
    beta = 0.5
    model = nn.AutoEncoder(grid=16, channels=(1, 8, 16, 32, 64), latent=64, dtype=torch.float64,
                           seed=7, vae_beta=beta)
    torch.manual_seed(8)
    with torch.no_grad():
        for k, p in model.params.items():
            if k.endswith(".b"):
                p.copy_(torch.randn(p.shape, dtype=torch.float64) * 0.1)
            if k == "enc_fc.w":
                p.mul_(0.3)
    x = torch.rand(2, 1, 16, 16, 16, dtype=torch.float64, device="cuda")
    eps = torch.randn(2, 64, dtype=torch.float64, device="cuda")

    def total():
        mse = nn.MSE.apply(model.forward(x, eps), x)
        return mse, float(mse.detach()) + beta * float(model.kl)

    mse, l0 = total()
    mse.backward()
    params_cpu = {k: p.detach().cpu() for k, p in model.params.items()}
    ref, _ = E.vae_loss(params_cpu, x.cpu(), eps.cpu(), beta, 64, 1)
    assert abs(l0 - float(ref)) <= 1e-12 * abs(float(ref))
    h = 1e-6
    rng = np.random.default_rng(9)
    checked = skipped = 0
    for name, p in model.params.items():
        g = p.grad.detach().cpu().numpy().ravel()
        flat = p.data.view(-1)
        coords = range(flat.numel()) if name.endswith(".b") else \
            rng.choice(flat.numel(), size=min(100, flat.numel()), replace=False)
        gmax = float(np.abs(g).max())
        for c in coords:
            c = int(c)
            old = float(flat[c])
            flat[c] = old + h
            lp = total()[1]
            flat[c] = old - h
            lm = total()[1]
            flat[c] = old
            fd = (lp - lm) / (2 * h)
            if abs((lp - l0) / h - (l0 - lm) / h) > 1e-3 * abs(fd) + 1e-6:
                skipped += 1
                continue
            assert abs(fd - g[c]) <= 1e-5 * abs(g[c]) + 1e-7 * gmax + 1e-9, (name, c, fd, g[c])
            checked += 1
    assert skipped <= 0.01 * (checked + skipped)
    say(f"VAE finite differences: {checked} coordinates agree, {skipped} skipped")
