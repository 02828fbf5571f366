"""GPU parity of the batched, box-restricted scan (one kernel launch replayed from a HIP graph).

Each query q is cut to its box R_q on both sides: I = |A n B n R|,
A = |A n R|, B = |B n R| (the paper compares whole volumes; the box is this
library's extension). Bar: bit-exact counts, score bits and indices.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI


def _host(t):
    return t.detach().cpu().numpy()


def _oracle_batch(conc, labels, rois, k):
    out = []
    for q in range(labels.shape[0]):
        roi = None if rois is None else rois[q]
        cnt, sc = oracle.scan_block(conc, labels[q], T_LO, T_HI, roi=roi)
        out.append((cnt, sc, oracle.rank(sc, k)))
    return out


def _compare(res, ref, k):
    idx, score, counts = (_host(t) for t in res)
    for q, (cnt, sc, top) in enumerate(ref):
        assert list(idx[q]) == top, f"query {q}"
        assert np.array_equal(score[q].view(np.uint64), sc[top].view(np.uint64)), f"query {q}"
        c = counts[q].view(np.uint32).astype(np.uint64)
        assert np.array_equal(c, cnt[top]), f"query {q}"


def _edge_rois(dims, nq, rng):
    nx, ny, nz = dims
    fixed = [
        (0, 0, 0, nx, ny, nz),              # whole grid
        (31, 3, 2, 33, 9, 7),               # spans a word boundary in x
        (5, 4, 3, 6, 5, 4),                 # single voxel
        (32, 0, 0, 64, ny, nz),             # word-aligned slab
        (nx - 1, ny - 1, nz - 1, nx, ny, nz),
        (1, 1, 1, nx - 1, ny - 1, nz - 1),
    ]
    rois = list(fixed)
    while len(rois) < nq:
        lo = [int(rng.integers(0, d)) for d in dims]
        hi = [int(rng.integers(l + 1, d + 1)) for l, d in zip(lo, dims)]
        rois.append((*lo, *hi))
    return np.array(rois[:nq], dtype=np.int32)


def test_batch_small_grid_parity():
    need_gpu()
    gen = synth.GenConfig(128, 24, 20, 2.0, 10.0, 0.5, 3.0, 31)
    n, nq, k = 203, 14, 10        # ragged tile count; k <= n
    say(f"batch: build n={n} on {gen.nx}x{gen.ny}x{gen.nz}")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    rng = np.random.default_rng(1)
    rois = _edge_rois((gen.nx, gen.ny, gen.nz), nq, rng)
    ref = _oracle_batch(conc, labels, rois, k)
    lab_d = torch.from_numpy(labels).cuda()
    ws = db.workspace(nq, k)
    out = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
           torch.empty((nq, k), dtype=torch.float64, device="cuda"),
           torch.empty((nq, k, 6), dtype=torch.int32, device="cuda"))
    # First call records the graph, later calls replay it; eager work in between.
    for rep in range(3):
        say(f"batch: replay {rep}")
        for t in out:
            t.fill_(-1)
        res = db.query_batch(lab_d, rois, k, out=out, ws=ws)
        db.sync()
        _compare(res, ref, k)
        _ = (lab_d.float().sum() + 1).item()
    # New boxes through the same graph (only the uploaded plan changes).
    rois2 = _edge_rois((gen.nx, gen.ny, gen.nz), nq, np.random.default_rng(2))[::-1].copy()
    ref2 = _oracle_batch(conc, labels, rois2, k)
    res = db.query_batch(lab_d, rois2, k, out=out, ws=ws)
    db.sync()
    _compare(res, ref2, k)


def test_batch_whole_grid_equals_single_query():
    need_gpu()
    gen = synth.SMALL
    n, nq, k = 300, 5, 10
    say("batch vs single")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    lab_d = torch.from_numpy(labels).cuda()
    bi, bs, bc = db.query_batch(lab_d, None, k)
    db.sync()
    for q in range(nq):
        si, ss, sc = db.query(lab_d[q], k)
        db.sync()
        assert torch.equal(bi[q], si) and torch.equal(bs[q], ss) and torch.equal(bc[q], sc)


def test_batch_boxes_of_the_workload_generator():
    need_gpu()
    gen = synth.SMALL
    n, nq, k = 256, 16, 10
    say("batch: workload-style boxes on 64^3")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    rois = synth.make_rois(labels, synth.ROI_SEED)
    ref = _oracle_batch(conc, labels, rois, k)
    res = db.query_batch(torch.from_numpy(labels).cuda(), rois, k)
    db.sync()
    _compare(res, ref, k)


def test_batch_results_do_not_depend_on_launch_shape():
    """Every launch shape the autotuner may pick (slab depth, block size, entries per tile,
    queries per chunk) and the kernel that reads the database through L2 (slab_planes
    = -1) give the same bytes."""
    need_gpu()
    gen = synth.GenConfig(128, 24, 20, 2.0, 10.0, 0.5, 3.0, 31)
    n, nq, k = 75, 9, 7
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    rois = _edge_rois((gen.nx, gen.ny, gen.nz), nq, np.random.default_rng(3))
    ref = _oracle_batch(conc, labels, rois, k)
    lab_d = torch.from_numpy(labels).cuda()
    for shape in [(0, 0, 0, 0), (1, 256, 4, 0), (2, 512, 8, 0), (3, 1024, 8, 4), (7, 512, 4, 2),
                  (20, 1024, 8, 1), (0, 1024, 8, 9), (-1, 0, 0, 0)]:
        say(f"shape planes, threads, tile, chunk = {shape}")
        db.tune_batch(*shape)
        res = db.query_batch(lab_d, rois, k)
        db.sync()
        _compare(res, ref, k)


@pytest.mark.parametrize("planes,tile", [(0, 4), (0, 8), (-1, 0)])
def test_batch_more_queries_than_one_chunk(planes, tile):
    """300 queries (more than the 256 of one query chunk: two chunks, each an item of the
    block per tile) with uneven boxes, against the oracle's loop over every entry;
    also through the kernel that reads the database through L2."""
    need_gpu()
    gen = synth.GenConfig(128, 24, 20, 2.0, 10.0, 0.5, 3.0, 37)
    n, nq, k = 61, 300, 5
    say(f"batch: {nq} queries, planes {planes}, tile {tile}")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    rois = _edge_rois((gen.nx, gen.ny, gen.nz), nq, np.random.default_rng(5))
    cnt, sc = oracle.scan_block_multi(conc, labels, T_LO, T_HI, rois)
    db.tune_batch(planes, 0, tile, 0)
    res = db.query_batch(torch.from_numpy(labels).cuda(), rois, k)
    db.sync()
    _compare(res, [(cnt[q], sc[q], oracle.rank(sc[q], k)) for q in range(nq)], k)
