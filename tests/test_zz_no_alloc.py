"""db_query_noalloc: the exact query with the library's fixed device scratch array.

Called through the C ABI and compared, bit for bit, with db_query (caller
workspace) and with the oracle, on two calls in a row where the second has a
smaller grid and database than the first (the scratch array keeps the first
call's bytes). A database whose workspace exceeds the array is refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI


def _noalloc(db, q, k):
    from paper_2205_04550_amd import binding as B
    idx = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    score = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
    counts = torch.full((k, 6), -1, dtype=torch.int32, device="cuda")
    rc = B.LIB.db_query_noalloc(db._h, ctypes.c_void_p(q.data_ptr()), k,
                                ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(score.data_ptr()),
                                ctypes.c_void_p(counts.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, idx, score, counts


def _check(db, conc, q, k):
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    rc, idx, score, counts = _noalloc(db, qd, k)
    assert rc == 0
    w_idx, w_score, w_counts = db.query(qd, k)
    torch.cuda.synchronize()
    assert torch.equal(idx, w_idx)
    assert np.array_equal(score.cpu().numpy().view(np.uint64), w_score.cpu().numpy().view(np.uint64))
    assert torch.equal(counts, w_counts)
    o_cnt, o_sc = oracle.scan_block(conc, q & 3, T_LO, T_HI)
    top = oracle.rank(o_sc, k)
    assert idx.cpu().tolist() == top
    assert np.array_equal(score.cpu().numpy().view(np.uint64), o_sc[top].view(np.uint64))
    assert np.array_equal(counts.cpu().numpy().view(np.uint32).astype(np.uint64), o_cnt[top])


def test_noalloc_query_equals_workspace_query_twice_shrinking():
    need_gpu()
    gen1, n1 = synth.SMALL, 300
    say(f"no-alloc: first call, {n1} x 64^3")
    db1, conc1 = build_db_from_host(gen1, n1, T_LO, T_HI)
    q1 = gen1.query(synth.query_source(n1, synth.QUERY_SEED, 0), T_LO, T_HI, synth.QUERY_SEED, 0)
    _check(db1, conc1, q1, 10)
    gen2 = synth.GenConfig(64, 16, 8, 1.0, 12.0, 0.5, 3.0, 31)
    n2 = 40
    say(f"no-alloc: second call, {n2} x 64x16x8, k = {n2}")
    db2, conc2 = build_db_from_host(gen2, n2, T_LO, T_HI)
    q2 = oracle.threshold(conc2[7], T_LO, T_HI)
    _check(db2, conc2, q2, n2)
    say("no-alloc: the first database again, k = 33")
    _check(db1, conc1, q1, 33)


def test_noalloc_refuses_a_database_beyond_the_scratch_array():
    need_gpu()
    from paper_2205_04550_amd import TumorDB, binding as B
    cap = 600_000                  # 8 bytes of overlaps per entry of capacity: 4.8 MB > 4 MiB
    say(f"no-alloc: capacity {cap} on 32x1x1 must be refused")
    db = TumorDB(32, 1, 1, cap, T_LO, T_HI)
    db.append(torch.linspace(0, 1, 32, device="cuda").reshape(1, 32))
    torch.cuda.synchronize()
    q = torch.ones(32, dtype=torch.uint8, device="cuda")
    rc, idx, score, counts = _noalloc(db, q, 1)
    assert rc == B.DB_ENOSPC
    assert b"scratch" in B.LIB.db_last_error()
    torch.cuda.synchronize()
    assert int(idx[0]) == -1 and float(score[0]) == -1.0 and bool((counts == -1).all())
    rc, *_ = _noalloc(db, q, 2)    # k > db_size()
    assert rc == B.DB_EINVAL
