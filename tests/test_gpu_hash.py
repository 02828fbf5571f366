"""GPU parity of the binary-code path (F3): thresholds, codes, Hamming distances,
candidate selection, exact rerank and the Bi-half layer, bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import oracle.encoder as E
import synth
from gpu_util import build_db_from_host, need_gpu, say

pytestmark = pytest.mark.gpu


def _h(t):
    return t.detach().cpu().numpy()


def test_thresholds_codes_and_hamming_exact():
    need_gpu()
    from paper_2205_04550_amd import binding as b
    rng = np.random.default_rng(8)
    for n, dim in ((50021, 512), (7, 32), (1000, 1024)):
        X = rng.standard_normal((n, dim)).astype(np.float32)
        X[:, 0] = np.round(X[:, 0])               # heavy ties in one coordinate
        X[: n // 3, 1] = -0.0                       # signed zeros
        say(f"hash: n={n} dim={dim}")
        Xd = torch.from_numpy(X).cuda()
        thr = b.hash_thresholds(Xd)
        want_thr = E.hash_thresholds(X)
        assert np.array_equal(_h(thr), want_thr)    # by value (+0 == -0)
        codes = b.BinaryCodes(Xd, thr)
        assert np.array_equal(_h(codes.codes).view(np.uint32), E.binarize(X, want_thr))
    # Hamming distances and their top-k (many equal integer distances: ties by index).
    Q = rng.standard_normal((37, 512)).astype(np.float32)
    X = rng.standard_normal((5003, 512)).astype(np.float32)
    thr = E.hash_thresholds(X)
    qc = b.BinaryCodes(torch.from_numpy(Q).cuda(), torch.from_numpy(thr).cuda())
    xc = b.BinaryCodes(torch.from_numpy(X).cuda(), torch.from_numpy(thr).cuda())
    D = b.emb_distances(qc, xc)
    want = E.hamming(E.binarize(Q, thr), E.binarize(X, thr))
    assert np.array_equal(_h(D), want)
    idx, val = b.emb_topk_min(D, 100)
    top = E.topk_by_distance(want, 100)
    assert np.array_equal(_h(idx), top)
    assert np.array_equal(_h(val), np.take_along_axis(want, top, 1))


def test_hash_query_chain_matches_oracle():
    """db_query_embed with binary codes: candidates by Hamming, exact rerank, as the oracle."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    gen = synth.SMALL
    n, nq, nc, k = 400, 5, 40, 10
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labs = np.stack([oracle.threshold(c, synth.T_LO, synth.T_HI) for c in conc])
    qs, _ = synth.make_queries(gen, n, nq, synth.QUERY_SEED)
    rng = np.random.default_rng(9)
    # Stand-in latents: any float rows work for the chain's parity.
    X = rng.standard_normal((n, 256)).astype(np.float32)
    Qf = X[: nq] + 0.3 * rng.standard_normal((nq, 256)).astype(np.float32)
    thr = E.hash_thresholds(X)
    xc = b.BinaryCodes(torch.from_numpy(X).cuda())
    qc = b.BinaryCodes(torch.from_numpy(Qf).cuda(), xc.thr)
    idx, score, counts, ci, cd = db.query_embed(b.EMB_BIN, qc, xc, torch.from_numpy(qs).cuda(), nc, k)
    db.sync()
    Dw = E.hamming(E.binarize(Qf, thr), E.binarize(X, thr))
    cand = E.topk_by_distance(Dw, nc)
    assert np.array_equal(_h(ci), cand)
    assert np.array_equal(_h(cd), np.take_along_axis(Dw, cand, 1))
    for j in range(nq):
        cnt = np.array([oracle.counts(qs[j], labs[e]) for e in cand[j]], dtype=np.uint64)
        sc = np.array([oracle.score(c) for c in cnt])
        order = oracle.rank(sc, k)
        assert _h(idx[j]).tolist() == [int(cand[j][o]) for o in order]
        assert np.array_equal(_h(score[j]).view(np.uint64), sc[order].view(np.uint64))
        assert np.array_equal(_h(counts[j]).view(np.uint32).astype(np.uint64), cnt[order])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_bihalf_layer_exact(dtype):
    need_gpu()
    from paper_2205_04550_amd import nn
    rng = np.random.default_rng(10)
    for B, D in ((32, 512), (33, 70), (2, 5)):
        U = rng.standard_normal((B, D)).astype(np.float64)
        U[:, 0] = np.round(U[:, 0])               # ties
        U = U.astype(np.float32 if dtype == torch.float32 else np.float64)
        G = rng.standard_normal((B, D)).astype(U.dtype)
        u = torch.from_numpy(U).cuda().requires_grad_(True)
        code = nn.BiHalf.apply(u, 3.0)
        code.backward(torch.from_numpy(G).cuda())
        Bc = E.bihalf_forward(U)
        assert np.array_equal(_h(code), Bc)
        assert np.array_equal(_h(u.grad), E.bihalf_backward(U, Bc, G, 3.0))
