"""Full-size parity: every entry of the 50,000 x 128^3 database against the oracle's loop.

The paper's ground truth is the exhaustive for-loop over the database
(Sec. 2.3, "Baseline for-loop search"). Here the oracle runs that loop over all
50,000 simulations, regenerated on the CPU chunk by chunk from the seeded
generator (419 GB of float32 in total, never held at once), for:
  - the single noisy query of the exact-scan workload: all 50,000 x 6 counts
    and the score bits of every entry against db_scan, and the top-10 of
    db_query against the oracle's full sort;
  - 8 of the 256 queries of one batched launch, each with its own box: the
    top-10 (indices, score bits, counts) of db_query_batch against the
    oracle's full sort over all 50,000 entries inside that box.
Bar: bit-exact. The GPU database is built on the GPU from the same generator
(its GPU build writes the CPU build's bytes; test_gpu_scan checks that).
"""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_on_gpu, need_gpu, say

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI
N_BATCH_CHECKED = 8


def _u64(t):
    return t.detach().cpu().numpy().view(np.uint32).astype(np.uint64)


@pytest.mark.timeout(1500)
def test_full_config_every_entry_against_the_oracle():
    need_gpu()
    gen, n, k = synth.FULL, synth.FULL_N, 10
    say("full parity: GPU-generated build of 50,000 x 128^3")
    db = build_db_on_gpu(gen, n, T_LO, T_HI, log=say)
    src = synth.query_source(n, synth.QUERY_SEED, 0)
    q = gen.query(src, T_LO, T_HI, synth.QUERY_SEED, 0)
    qd = torch.from_numpy(q).cuda()
    say("full parity: single query (db_query, db_scan)")
    idx, score, counts = db.query(qd, k)
    inter, qcount = db.scan(qd)
    say("full parity: 256 box-restricted queries in one batched launch")
    labels, _ = synth.make_queries(gen, n, 256, synth.BATCH_QUERY_SEED)
    rois = synth.make_rois(labels, synth.ROI_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    bidx, bscore, bcounts = db.query_batch(lab_d, rois, k)
    db.sync()
    inter, a = _u64(inter), _u64(qcount)
    pcs = _u64(db.popcounts)[:n]
    idx, score, counts = idx.cpu().numpy(), score.cpu().numpy(), _u64(counts)
    bidx, bscore, bcounts = bidx.cpu().numpy(), bscore.cpu().numpy(), _u64(bcounts)
    del lab_d, db
    torch.cuda.empty_cache()
    # Queries checked from the batch: spread over the box volumes, smallest and largest included.
    vol = np.prod(rois[:, 3:6] - rois[:, 0:3], axis=1)
    by_vol = np.argsort(vol, kind="stable")
    pick = sorted(set(by_vol[np.linspace(0, 255, N_BATCH_CHECKED).round().astype(int)].tolist()))
    Q = np.concatenate([q[None], labels[pick]])
    R = np.concatenate([np.array([[0, 0, 0, gen.nx, gen.ny, gen.nz]], np.int32), rois[pick]])
    del labels
    threads = oracle._threads()
    say(f"full parity: oracle loop over all {n} entries x {len(Q)} queries on {threads} threads")
    o_cnt = np.zeros((len(Q), n, 6), np.uint64)
    o_sc = np.zeros((len(Q), n), np.float64)
    chunk, t0, gen_s = 512, time.perf_counter(), 0.0
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        tg = time.perf_counter()
        conc = gen.conc_cpu(s, c, threads)
        gen_s += time.perf_counter() - tg
        o_cnt[:, s:s + c], o_sc[:, s:s + c] = oracle.scan_block_multi(conc, Q, T_LO, T_HI, R,
                                                                      threads)
        if (s // chunk) % 10 == 0:
            say(f"  oracle {s + c}/{n} entries, {time.perf_counter() - t0:.0f} s "
                f"({gen_s:.0f} s generating)")
    del conc
    say(f"full parity: oracle done in {time.perf_counter() - t0:.0f} s")
    # Single query: every count and every score.
    assert np.array_equal(inter, o_cnt[0, :, 0:2])
    assert np.array_equal(pcs, o_cnt[0, :, 4:6])
    assert (int(a[0]), int(a[1])) == (int(o_cnt[0, 0, 2]), int(o_cnt[0, 0, 3]))
    implied = np.array([oracle.score((inter[e, 0], inter[e, 1], a[0], a[1], pcs[e, 0], pcs[e, 1]))
                        for e in range(n)])
    assert np.array_equal(implied.view(np.uint64), o_sc[0].view(np.uint64))
    top = oracle.rank(o_sc[0], k)
    assert list(idx) == top
    assert np.array_equal(score.view(np.uint64), o_sc[0][top].view(np.uint64))
    assert np.array_equal(counts, o_cnt[0][top])
    say(f"full parity: single query ok; source {src} at rank "
        f"{top.index(src) if src in top else '>10'}")
    # Batched queries: top-10 of each against the full sort inside its box.
    for j, qi in enumerate(pick):
        topj = oracle.rank(o_sc[j + 1], k)
        assert list(bidx[qi]) == topj, (qi, list(bidx[qi]), topj)
        assert np.array_equal(bscore[qi].view(np.uint64), o_sc[j + 1][topj].view(np.uint64))
        assert np.array_equal(bcounts[qi], o_cnt[j + 1][topj])
    say(f"full parity: batched queries {pick} ok (box volumes {vol[pick].tolist()})")
