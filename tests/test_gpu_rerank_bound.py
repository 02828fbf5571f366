"""GPU checks of the bound-ordered rerank (candidates scored in decreasing order of a bound on
their Dice score, those that cannot reach the top k left out): the per-entry 16^3-block counts
equal those of the oracle's masks; every entry's bound is at least its exact score; the top k,
scores and counts equal those of scoring every candidate and the oracle's, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say

pytestmark = pytest.mark.gpu

GRIDS = {
    "64cube": synth.SMALL,
    "128cube": synth.FULL,
    "ragged": synth.GenConfig(96, 40, 24, 3.0, 12.0, 0.5, 3.0, synth.DB_SEED),  # partial blocks
}


def _blocks(mask: np.ndarray) -> np.ndarray:
    """Set voxels per 16^3 block of bool masks [..][nz][ny][nx], flattened (bz, by, bx)."""
    *lead, nz, ny, nx = mask.shape
    pz, py, px = -nz % 16, -ny % 16, -nx % 16
    m = np.pad(mask, [(0, 0)] * len(lead) + [(0, pz), (0, py), (0, px)])
    bz, by, bx = m.shape[-3] // 16, m.shape[-2] // 16, m.shape[-1] // 16
    m = m.reshape(*lead, bz, 16, by, 16, bx, 16)
    return m.sum(axis=(-5, -3, -1), dtype=np.int64).reshape(*lead, bz * by * bx)


def _setup(name, n, nq, seed):
    gen = GRIDS[name]
    say(f"bound rerank {name}: build {n}")
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labels, _ = synth.make_queries(gen, n, nq, seed)
    return gen, db, conc, labels


@pytest.mark.parametrize("name,n", [("64cube", 300), ("128cube", 60), ("ragged", 200)])
def test_block_counts_and_bound_at_least_score(name, n):
    need_gpu()
    gen, db, conc, labels = _setup(name, n, 4, synth.BATCH_QUERY_SEED)
    nbx, nby, nbz, nbp = db.block_dims()
    assert nbp and nbp % 8 == 0 and nbp >= nbx * nby * nbz
    lab = oracle.threshold(conc, synth.T_LO, synth.T_HI)
    want = np.stack([_blocks((lab & 1) != 0), _blocks((lab & 2) != 0)], axis=1)   # [n][2][nb]
    got = db.block_counts[:n].cpu().numpy().view(np.uint16).astype(np.int64)
    nb = nbx * nby * nbz
    assert np.array_equal(got[:, :, :nb], want)
    assert not got[:, :, nb:].any()
    for q in range(labels.shape[0]):
        cnt, sc = oracle.scan_block(conc, labels[q], synth.T_LO, synth.T_HI)
        qb = np.stack([_blocks((labels[q] & 1) != 0), _blocks((labels[q] & 2) != 0)])
        ub = np.minimum(want, qb[None]).sum(axis=2)                                # [n][2]
        aF, aT = int((labels[q] & 1).astype(bool).sum()), int((labels[q] & 2).astype(bool).sum())
        bF, bT = want[:, 0].sum(1), want[:, 1].sum(1)
        bound = np.array([oracle.dice(int(ub[e, 1]), aT, int(bT[e])) +
                          oracle.dice(int(ub[e, 0]), aF, int(bF[e])) for e in range(n)])
        assert (bound >= sc).all(), (q, float((sc - bound).max()))


@pytest.mark.parametrize("name,n,nc", [("64cube", 300, 17), ("64cube", 300, 100),
                                       ("64cube", 300, 300), ("128cube", 60, 40),
                                       ("ragged", 200, 100)])
def test_bound_rerank_equals_scoring_every_candidate(name, n, nc):
    need_gpu()
    gen, db, conc, labels = _setup(name, n, 8, synth.QUERY_SEED)
    nq = labels.shape[0]
    labels[3] = 0                                                  # an empty query
    rng = np.random.default_rng(n + nc)
    cand = np.empty((nq, nc), dtype=np.int32)
    full = []
    for q in range(nq):
        cnt, sc = oracle.scan_block(conc, labels[q], synth.T_LO, synth.T_HI)
        full.append((cnt, sc))
        if q % 2:                                                  # the nearest, as a search gives
            cand[q] = sorted(range(n), key=lambda e: (-sc[e], e))[:nc]
        else:
            cand[q] = rng.choice(n, nc, replace=False)
    lab_d = torch.from_numpy(labels).cuda()
    cand_d = torch.from_numpy(cand).cuda()
    for k in (1, 10, 15, 33, 64, min(nc, 100)):
        if k > nc:
            continue
        db.set_rerank_bound(False)
        fi, fs, fc = db.rerank(lab_d, cand_d, k)
        db.set_rerank_bound(True)
        bi, bs, bc = db.rerank(lab_d, cand_d, k)
        db.sync()
        assert torch.equal(bi, fi) and torch.equal(bs.view(torch.int64), fs.view(torch.int64)), k
        assert torch.equal(bc, fc), k
        for q in range(nq):
            cnt, sc = full[q]
            order = sorted(range(nc), key=lambda j: (-sc[cand[q][j]], cand[q][j]))[:k]
            assert bi[q].cpu().tolist() == [int(cand[q][j]) for j in order], (k, q)
            assert np.array_equal(bs[q].cpu().numpy().view(np.uint64),
                                  sc[cand[q][order]].view(np.uint64)), (k, q)
