"""GPU parity of the row-box metadata, the box-restricted exact scan and the
centre-of-mass prefilter (F2): bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, build_db_on_gpu, need_gpu, say

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI


def _host(t):
    return t.detach().cpu().numpy()


def _edge_queries(gen, labs, rng):
    """Noisy entries, an empty query, a T1Gd-only query, a whole-grid query and a
    single-voxel query."""
    shape = (gen.nz, gen.ny, gen.nx)
    qs, _ = synth.make_queries(gen, len(labs), 3, synth.QUERY_SEED)
    extra = [np.zeros(shape, np.uint8), (labs[1] & 2), np.full(shape, 3, np.uint8),
             np.zeros(shape, np.uint8)]
    extra[3][gen.nz // 2, gen.ny - 1, gen.nx - 1] = 3
    return list(qs) + extra


@pytest.mark.parametrize("dims", [(128, 64, 48), (64, 64, 64), (96, 40, 30)])
def test_meta_and_sparse_query_match_oracle(dims):
    need_gpu()
    gen = synth.GenConfig(*dims, 2.0, max(4.0, dims[0] / 6), 0.5, 3.0, 43)
    n, k = 60, 12
    say(f"sparse: {dims} x {n}")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labs = np.stack([oracle.threshold(c, T_LO, T_HI) for c in conc])
    # An entry with no set bit, and one that fills the whole grid.
    conc2 = np.zeros((2,) + conc.shape[1:], np.float32)
    conc2[1] = 1.0
    db2, _ = build_db_from_host(gen, n + 2, T_LO, T_HI, conc=np.concatenate([conc, conc2]))
    labs2 = np.concatenate([labs, np.stack([oracle.threshold(c, T_LO, T_HI) for c in conc2])])
    for d, L in ((db, labs), (db2, labs2)):
        boxes = _host(d.boxes)[:len(L)]
        tboxes = _host(d.tboxes)[:len(L)]
        zr = _host(d.zranges)[:len(L)].view(np.uint32)
        moms = _host(d.moments)[:len(L)].view(np.uint64)
        for i in range(len(L)):
            assert tuple(boxes[i]) == oracle.rowbox(L[i]), i
            assert tuple(tboxes[i]) == oracle.rowbox(L[i] & 2), i      # the T1Gd rows alone
            # Per z-slice: [y0, y1) of the rows holding a FLAIR bit, and of those holding a T1Gd
            # bit, packed y0 | y1 << 16 (0 for a slice without any).
            for p, bit in ((0, 1), (1, 2)):
                rows = ((L[i] & bit) != 0).any(axis=2)                  # [nz][ny]
                want = np.zeros(L[i].shape[0], np.uint32)
                for z in np.nonzero(rows.any(axis=1))[0]:
                    ys = np.nonzero(rows[z])[0]
                    want[z] = int(ys.min()) | (int(ys.max()) + 1) << 16
                assert np.array_equal(zr[i, :, p], want), (i, p)
            assert tuple(int(v) for v in moms[i]) == oracle.moments(L[i]), i
    rng = np.random.default_rng(3)
    for j, q in enumerate(_edge_queries(gen, labs2, rng)):
        qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
        cnt = np.array([oracle.counts(q, L) for L in labs2], dtype=np.uint64)
        sc = np.array([oracle.score(c) for c in cnt])
        top = oracle.rank(sc, k)
        idx, score, counts = db2.query_sparse(qd, k)
        db2.sync()
        assert _host(idx).tolist() == top, j
        assert np.array_equal(_host(score).view(np.uint64), sc[top].view(np.uint64)), j
        assert np.array_equal(_host(counts).view(np.uint32).astype(np.uint64), cnt[top]), j


def test_com_prefilter_matches_oracle():
    need_gpu()
    gen = synth.GenConfig(128, 64, 48, 2.0, 12.0, 0.5, 3.0, 47)
    n = 300
    say(f"com: {n} entries")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labs = np.stack([oracle.threshold(c, T_LO, T_HI) for c in conc])
    qs, _ = synth.make_queries(gen, n, 4, synth.QUERY_SEED)
    empty = np.zeros_like(qs[:1])
    qs = np.concatenate([qs, empty])
    qd = torch.from_numpy(qs).cuda()
    for n_cand, k in ((50, 10), (n, 15)):
        idx, score, counts, ci, cd = db.query_com(qd, n_cand, k)
        db.sync()
        for j in range(len(qs)):
            cand, keys, top, sc, cnt = oracle.query_com(qs[j], labs, n_cand, k)
            assert _host(ci[j]).tolist() == cand.tolist(), (n_cand, j)
            assert np.array_equal(_host(cd[j]).view(np.uint32), keys.view(np.uint32)), (n_cand, j)
            assert _host(idx[j]).tolist() == top.tolist(), (n_cand, j)
            assert np.array_equal(_host(score[j]).view(np.uint64), sc.view(np.uint64))
            assert np.array_equal(_host(counts[j]).view(np.uint32).astype(np.uint64), cnt)


def test_full_size_sparse_equals_dense_and_oracle():
    """50,000 x 128^3: the sparse query returns the dense query's results for the
    benchmark's queries, and the oracle recomputes the returned entries."""
    need_gpu()
    gen, n, k = synth.FULL, synth.FULL_N, 10
    say("full config: GPU-generated build of 50,000 x 128^3")
    db = build_db_on_gpu(gen, n, T_LO, T_HI, log=say)
    # Box and moments of sampled entries against the oracle on regenerated volumes.
    rng = np.random.default_rng(7)
    sample = sorted(rng.choice(n, 12, replace=False).tolist())
    boxes = _host(db.boxes)
    moms = _host(db.moments).view(np.uint64)
    for e in sample:
        L = oracle.threshold(gen.conc_cpu(e, 1)[0], T_LO, T_HI)
        assert tuple(boxes[e]) == oracle.rowbox(L)
        assert tuple(int(v) for v in moms[e]) == oracle.moments(L)
    qs, srcs = synth.make_queries(gen, n, 4, synth.QUERY_SEED)
    for j in range(len(qs)):
        qd = torch.from_numpy(qs[j]).cuda()
        a = db.query(qd, k)
        b = db.query_sparse(qd, k)
        db.sync()
        for x, y in zip(a, b):
            assert torch.equal(x, y), j
        top = _host(a[0]).tolist()
        _, o_cnt, o_sc = oracle.scan(gen, n, qs[j], T_LO, T_HI, indices=top)
        assert np.array_equal(_host(b[2]).view(np.uint32).astype(np.uint64), o_cnt)
        assert np.array_equal(_host(b[1]).view(np.uint64), o_sc.view(np.uint64))
        say(f"full config: query {j} (source {srcs[j]}) -> {top[:3]}")
