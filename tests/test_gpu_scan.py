"""GPU parity of the exact scan (threshold + pack, AND+popcount, Dice, top-k) against the oracle.

Bar: bit-exact. Integer counts and indices must be equal; Dice and score are
compared as IEEE double bit patterns (both sides compute 2I/(A+B) and the
two-term sum in double with correct rounding).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say, unpack_planes

pytestmark = pytest.mark.gpu

T_LO, T_HI = synth.T_LO, synth.T_HI


def _host(t):
    return t.detach().cpu().numpy()


def _check_topk_against_oracle(idx, score, counts, o_cnt, o_sc, k):
    top = oracle.rank(o_sc, k)
    assert list(_host(idx)) == top
    assert np.array_equal(_host(score).view(np.uint64), o_sc[top].view(np.uint64))
    if counts is not None:
        c = _host(counts).view(np.uint32).astype(np.uint64)  # inter0, inter1, a0, a1, b0, b1
        assert np.array_equal(c, o_cnt[top])


def test_gpu_generator_writes_the_cpu_bytes():
    need_gpu()
    for gen, n0, n in ((synth.SMALL, 0, 6), (synth.FULL, 1234, 2)):
        say(f"generator {gen.nx}^3 n0={n0} n={n}")
        p = torch.from_numpy(gen.params(n0, n).view(np.float64).reshape(n, 8).copy()).cuda()
        out = torch.empty((n, gen.nvox), dtype=torch.float32, device="cuda")
        gen.conc_gpu(p.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        ref = gen.conc_cpu(n0, n).reshape(n, -1)
        got = _host(out)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("dims", [(64, 64, 64), (96, 5, 3), (32, 1, 1)])
def test_pack_matches_oracle_threshold(dims):
    need_gpu()
    nx, ny, nz = dims
    gen = synth.GenConfig(nx, ny, nz, 1.0, max(2.0, nx / 4), 0.5, 3.0, 77)
    n = 24
    say(f"pack dims={dims} n={n}")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI, capacity=n + 3)
    V = nx * ny * nz
    planes = _host(db.planes)[:n]                 # [n][2][Wp]
    pcs = _host(db.popcounts)[:n].view(np.uint32)
    bits = unpack_planes(planes, db.Wp * 32)
    for i in range(n):
        lab = oracle.threshold(conc[i], T_LO, T_HI).reshape(-1)
        for m in range(2):
            want = ((lab >> m) & 1).astype(bool)
            assert np.array_equal(bits[i, m, :V], want)
            assert not bits[i, m, V:].any()      # padding words are zero
            assert int(pcs[i, m]) == int(want.sum())
    assert len(db) == n


def test_small_config_full_parity():
    """1,000 sims on 64^3 with a noisy self-query, top-10; every count compared."""
    need_gpu()
    gen, n, k = synth.SMALL, synth.SMALL_N, 10
    say("small config: generate + build")
    db, conc = build_db_from_host(gen, n, T_LO, T_HI)
    src = synth.query_source(n, synth.QUERY_SEED, 0)
    q = gen.query(src, T_LO, T_HI, synth.QUERY_SEED, 0)
    o_cnt, o_sc = oracle.scan_block(conc, q, T_LO, T_HI)
    qd = torch.from_numpy(q).cuda()
    inter, qcount = db.scan(qd)
    torch.cuda.synchronize()
    assert np.array_equal(_host(inter).view(np.uint32).astype(np.uint64), o_cnt[:, 0:2])
    assert list(_host(qcount)) == [int(o_cnt[0, 2]), int(o_cnt[0, 3])]
    assert np.array_equal(_host(db.popcounts)[:n].view(np.uint32).astype(np.uint64), o_cnt[:, 4:6])
    for kk in (1, k, 32, 33, 333, n):   # 32 / 33: the two selection paths
        say(f"small config: query k={kk}")
        idx, score, counts = db.query(qd, kk)
        db.sync()
        _check_topk_against_oracle(idx, score, counts, o_cnt, o_sc, kk)
    # Repeated calls give identical bytes.
    a = db.query(qd, k)
    b = db.query(qd, k)
    db.sync()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_ragged_grid_ties_and_empty_query():
    need_gpu()
    gen = synth.GenConfig(96, 5, 3, 1.0, 20.0, 0.5, 3.0, 99)
    base = gen.conc_cpu(0, 30)
    # Entries 30..36 duplicate entries 4 and 9: equal scores resolve to the lower index.
    conc = np.concatenate([base, base[[4, 4, 9, 9, 4, 9, 4]]])
    n = conc.shape[0]
    say(f"ragged grid n={n}")
    db, _ = build_db_from_host(gen, n, T_LO, T_HI, conc=conc, capacity=64, chunk=16)
    rng = np.random.default_rng(0)
    queries = [oracle.threshold(conc[4], T_LO, T_HI),
               np.zeros(conc.shape[1:], np.uint8),
               rng.integers(0, 4, size=conc.shape[1:], dtype=np.uint8),
               (rng.integers(0, 256, size=conc.shape[1:])).astype(np.uint8)]  # high bits ignored
    for qi, q in enumerate(queries):
        o_cnt, o_sc = oracle.scan_block(conc, q & 3, T_LO, T_HI)
        qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
        for k in (1, 5, n):
            say(f"  query {qi} k={k}")
            idx, score, counts = db.query(qd, k)
            db.sync()
            _check_topk_against_oracle(idx, score, counts, o_cnt, o_sc, k)
    # Self-query of entry 4 scores exactly 2 for 4 and its duplicates, lowest index first.
    idx, score, _ = db.query(torch.from_numpy(queries[0]).cuda(), 5)
    db.sync()
    assert list(_host(idx)) == [4, 30, 31, 34, 36]
    assert list(_host(score)) == [2.0] * 5


def test_selection_levels_with_ties_across_blocks():
    """70,000 entries (69 selection blocks of 1,024): k = 32 takes three levels, k = 33
    the LDS path; entries drawn with repetition from 700 volumes, so equal scores fall in
    different blocks and levels and must still come out lowest index first."""
    need_gpu()
    gen = synth.GenConfig(32, 4, 4, 1.0, 6.0, 0.5, 2.0, 5)
    rng = np.random.default_rng(11)
    conc = gen.conc_cpu(0, 700)[rng.integers(0, 700, size=70_000)]
    n = conc.shape[0]
    say(f"selection levels n={n}")
    db, _ = build_db_from_host(gen, n, T_LO, T_HI, conc=conc, chunk=8192)
    for qi, q in enumerate((oracle.threshold(conc[123], T_LO, T_HI),
                            rng.integers(0, 4, size=conc.shape[1:], dtype=np.uint8))):
        o_cnt, o_sc = oracle.scan_block(conc, q, T_LO, T_HI)
        qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
        for k in (1, 10, 32, 33, 500):
            say(f"  query {qi} k={k}")
            idx, score, counts = db.query(qd, k)
            db.sync()
            _check_topk_against_oracle(idx, score, counts, o_cnt, o_sc, k)


def test_errors_write_nothing():
    need_gpu()
    from paper_2205_04550_amd import DbError, binding
    gen = synth.GenConfig(64, 8, 8, 1.0, 10.0, 0.5, 3.0, 5)
    db, conc = build_db_from_host(gen, 12, T_LO, T_HI, capacity=12)
    qd = torch.zeros((8, 8, 64), dtype=torch.uint8, device="cuda")
    idx = torch.full((20,), -7, dtype=torch.int32, device="cuda")
    score = torch.full((20,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(DbError) as e:
        db.query(qd, 13, out=(idx, score, None))       # k > N
    assert e.value.code == binding.DB_EINVAL
    small_ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(DbError) as e:
        db.query(qd, 3, out=(idx, score, None), ws=small_ws)
    assert e.value.code == binding.DB_ENOSPC
    with pytest.raises(DbError) as e:
        db.append(torch.from_numpy(conc[:1]).cuda())   # over capacity
    assert e.value.code == binding.DB_ENOSPC
    with pytest.raises(DbError) as e:
        db.query_batch(qd[None], [[0, 0, 0, 65, 8, 8]], 3)  # box outside the grid
    assert e.value.code == binding.DB_EINVAL
    with pytest.raises(DbError):
        db.query_batch(qd[None], [[5, 0, 0, 5, 8, 8]], 3)   # empty box
    torch.cuda.synchronize()
    assert bool((idx == -7).all()) and bool((score == -7.0).all())
    assert len(db) == 12
