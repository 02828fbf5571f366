"""GPU parity of the downsampled exact scan (DS64 / DS32, paper Sec. 2.3): order-0
resampling of the packed masks and of the query labels, then the same exact query.
Bar: bit-exact against scipy's order-0 zoom of the oracle's thresholded volumes."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say, unpack_planes

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI


@pytest.mark.parametrize("src,dst", [((128, 64, 48), (64, 32, 24)), ((128, 64, 48), (32, 16, 12)),
                                     ((64, 64, 64), (32, 21, 7))])
def test_resampled_database_and_query_match_scipy(src, dst):
    need_gpu()
    from paper_2205_04550_amd import TumorDB
    from paper_2205_04550_amd.binding import labels_resample
    gen = synth.GenConfig(*src, 2.0, max(4.0, src[0] / 6), 0.5, 3.0, 41)
    n = 40
    say(f"resample {src} -> {dst}")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    nx, ny, nz = dst
    ds = TumorDB(nx, ny, nz, n, T_LO, T_HI)
    ds.append_resampled(db, 0, 25)
    ds.append_resampled(db, 25, 15)          # two appends: ragged chunks
    torch.cuda.synchronize()
    labs = np.stack([oracle.threshold(c, T_LO, T_HI) for c in conc])
    want = oracle.resample_nearest(labs, (nz, ny, nx))
    V = nx * ny * nz
    bits = unpack_planes(ds.planes.cpu().numpy()[:n], ds.Wp * 32)
    pcs = ds.popcounts.cpu().numpy()[:n].view(np.uint32)
    for i in range(n):
        for m in range(2):
            w = ((want[i].reshape(-1) >> m) & 1).astype(bool)
            assert np.array_equal(bits[i, m, :V], w)
            assert int(pcs[i, m]) == int(w.sum())
    # Queries: labels resampled on the device equal scipy's; the query on the small
    # database equals the oracle's loop on the resampled volumes.
    q, _ = synth.make_queries(gen, n, 3, synth.QUERY_SEED)
    qd = labels_resample(torch.from_numpy(q).cuda(), (nz, ny, nx))
    qw = oracle.resample_nearest(q, (nz, ny, nx))
    assert np.array_equal(qd.cpu().numpy(), qw)
    for j in range(3):
        cnt = np.array([oracle.counts(qw[j], want[i]) for i in range(n)], dtype=np.uint64)
        sc = np.array([oracle.score(c) for c in cnt])
        top = oracle.rank(sc, 10)
        idx, score, counts = ds.query(qd[j], 10)
        ds.sync()
        assert idx.cpu().tolist() == top
        assert np.array_equal(score.cpu().numpy().view(np.uint64), sc[top].view(np.uint64))
        assert np.array_equal(counts.cpu().numpy().view(np.uint32).astype(np.uint64), cnt[top])
