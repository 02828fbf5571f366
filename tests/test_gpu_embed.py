"""GPU parity of the embedding search: quantisation (bit-exact), MFMA distances (within
1e-5 of |q|^2 + |x|^2 against float64 direct form), exact top-k selection, and exact
Dice rerank of the candidates (bit-exact against the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import build_db_from_host, need_gpu, say
from oracle import encoder as E

pytestmark = pytest.mark.gpu


def _lat(n, dim, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(n, dim, generator=g) * scale).to(torch.float32)


def _dequant(L):
    from paper_2205_04550_amd import binding as b
    if L.fmt == b.EMB_BF16:
        return E.bf16_decode(L.codes.view(torch.int16).cpu().numpy())
    return E.e4m3_decode(L.codes.cpu().numpy()) * L.scale.cpu().numpy().astype(np.float64)[:, None]


@pytest.mark.parametrize("fmt", [0, 1])
def test_quantisation_bit_exact(fmt):
    need_gpu()
    from paper_2205_04550_amd import binding as b
    lat = _lat(37, 128, 1)
    lat[3] = 0.0                                   # zero row: scale 1, all codes zero
    lat[5, :7] = torch.tensor([448.0, -1e-9, 3e-3, 1e-8, -0.0, 7.0, -3.5])
    L = b.Latents(lat.cuda(), fmt)
    torch.cuda.synchronize()
    x = lat.numpy()
    if fmt == b.EMB_BF16:
        assert np.array_equal(L.codes.view(torch.int16).cpu().numpy().view(np.uint16), E.bf16_encode(x))
    else:
        amax = np.abs(x).max(axis=1)
        s = np.where(amax > 0, (amax / np.float32(448.0)).astype(np.float32), np.float32(1.0))
        assert np.array_equal(L.scale.cpu().numpy(), s)
        want = np.stack([E.e4m3_encode((x[i] / s[i]).astype(np.float32)) for i in range(x.shape[0])])
        assert np.array_equal(L.codes.cpu().numpy(), want)
    deq = _dequant(L)
    sq = (deq ** 2).sum(axis=1)
    assert np.allclose(L.sq.cpu().numpy(), sq, rtol=2e-7, atol=0)


@pytest.mark.parametrize("fmt,dim", [(0, 512), (0, 48), (1, 512), (1, 64)])
def test_distances_within_contract(fmt, dim):
    need_gpu()
    from paper_2205_04550_amd import binding as b
    M, N = 77, 1301                                  # ragged against the 128 x 128 tiles
    Q = b.Latents(_lat(M, dim, 2).cuda(), fmt)
    X = b.Latents(torch.cat([_lat(M, dim, 2)[:5], _lat(N - 5, dim, 3)]).cuda(), fmt)  # 5 self-pairs
    D = b.emb_distances(Q, X).cpu().numpy().astype(np.float64)
    q, x = _dequant(Q), _dequant(X)
    d64 = E.sqdist_direct(q, x)
    # The 1e-5 contract for both formats (FP8 codes are decoded exactly to BF16).
    rel = 1e-5
    bound = rel * ((q ** 2).sum(1)[:, None] + (x ** 2).sum(1)[None, :])
    err = np.abs(D - d64)
    say(f"fmt {fmt} dim {dim}: max |d - d64| / bound = {(err / bound).max():.3g}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("fmt,M,N,dim", [(0, 300, 50_021, 512), (1, 300, 50_021, 512),
                                         (0, 3, 1_100_000, 1024)])
def test_distances_many_tiles_and_chunks(fmt, M, N, dim):
    """Many tiles per block of the persistent grid, a ragged last query tile, and (BF16,
    dim 1024, 1.1M rows = 2.25 GB of codes) a database taken in two chunks: sampled
    columns (both ends, the chunk boundary at row 1,048,320, random) within the contract."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    g = torch.Generator(device="cuda").manual_seed(31)
    Qf = torch.randn(M, dim, generator=g, device="cuda")
    Xf = torch.randn(N, dim, generator=g, device="cuda")
    Q, X = b.Latents(Qf, fmt), b.Latents(Xf, fmt)
    del Xf
    D = b.emb_distances(Q, X)
    rng = np.random.default_rng(3)
    cols = np.unique(np.concatenate([np.arange(200), np.arange(N - 300, N),
                                     np.arange(1_048_320 - 64, 1_048_320 + 64) if N > 1_048_384
                                     else np.arange(0),
                                     rng.integers(0, N, 500)]))
    cols_d = torch.from_numpy(cols).cuda()
    class Sub:                                    # the sampled database rows, as Latents
        pass
    xs = Sub()
    xs.fmt, xs.codes = fmt, X.codes[cols_d].cpu()
    xs.scale = X.scale[cols_d].cpu() if X.scale is not None else None
    q, x = _dequant(Q), _dequant(xs)
    d64 = E.sqdist_direct(q, x)
    got = D[:, cols_d].cpu().numpy().astype(np.float64)
    rel = 1e-5
    bound = rel * ((q ** 2).sum(1)[:, None] + (x ** 2).sum(1)[None, :])
    say(f"fmt {fmt} {M} x {N} x {dim}: max |d - d64| / bound = {(np.abs(got - d64) / bound).max():.3g}")
    assert np.all(np.abs(got - d64) <= bound)


@pytest.mark.parametrize("fmt,M,N,dim,ks", [
    (0, 9, 50_021, 64, (1, 10, 100, 1000)),     # ragged N (not a multiple of 4 or 16)
    (1, 9, 50_021, 64, (1, 10, 100)),
    (0, 5, 3000, 48, (7, 100)),                 # k too large for a bound: one block per row
    (0, 4, 300_000, 64, (1, 7, 100)),           # 8,192-entry chunks
    (1, 3, 10, 64, (1, 5)),                      # fewer entries than one group
])
def test_groups_path_equals_plain_path(fmt, M, N, dim, ks):
    """emb_distances_groups writes the same D as emb_distances, and emb_topk_groups gives
    emb_topk_min's indices and values bit for bit: database rows repeated (exact ties
    across groups and chunks), one query equal to a database row, and one database of
    identical rows (every distance equal: the gather overflows and the row is selected
    by the one-block path)."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    g = torch.Generator(device="cuda").manual_seed(17)
    base = torch.randn(701, dim, generator=g, device="cuda")
    Xf = base.repeat(N // 701 + 1, 1)[:N].contiguous()
    Qf = torch.randn(M, dim, generator=g, device="cuda")
    Qf[1] = base[3]
    for Xlat in (Xf, base[:1].repeat(N, 1)):
        Q, X = b.Latents(Qf, fmt), b.Latents(Xlat, fmt)
        D0 = b.emb_distances(Q, X)
        ws = b.groups_workspace(M, N)
        D1 = b.emb_distances_groups(Q, X, ws)
        assert torch.equal(D0.view(torch.int32), D1.view(torch.int32))
        for k in ks:
            i0, v0 = b.emb_topk_min(D0, k)
            i1, v1 = b.emb_topk_groups(D1, k, ws)
            assert torch.equal(i0, i1) and torch.equal(v0.view(torch.int32), v1.view(torch.int32)), k
        want = E.topk_by_distance(D0.cpu().numpy(), ks[-1])
        assert np.array_equal(i1.cpu().numpy(), want)


def test_groups_path_chunked_database():
    """A BF16 database of 2.25 GB of codes (two launches of the distance kernel): group
    minima written at the right offsets on both sides of the chunk boundary."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    g = torch.Generator(device="cuda").manual_seed(23)
    N = 1_100_000
    Xf = torch.randn(N, 1024, generator=g, device="cuda")
    Qf = torch.randn(3, 1024, generator=g, device="cuda")
    Qf[2] = Xf[1_048_330]                         # its nearest entry just past the boundary
    Q, X = b.Latents(Qf, 0), b.Latents(Xf, 0)
    del Xf
    D0 = b.emb_distances(Q, X)
    ws = b.groups_workspace(3, N)
    D1 = b.emb_distances_groups(Q, X, ws)
    assert torch.equal(D0.view(torch.int32), D1.view(torch.int32))
    i0, v0 = b.emb_topk_min(D0, 10)
    i1, v1 = b.emb_topk_groups(D1, 10, ws)
    assert torch.equal(i0, i1) and torch.equal(v0, v1)
    assert int(i1[2, 0]) == 1_048_330


def test_topk_min_exact_with_ties():
    need_gpu()
    from paper_2205_04550_amd import binding as b
    rng = np.random.default_rng(4)
    M, N = 9, 50021
    D = rng.integers(0, 500, size=(M, N)).astype(np.float32) * np.float32(0.25)  # many ties
    D[2] = 7.0                                                   # a row of equal values
    D[3, 100:110] = -1.5                                         # negatives
    Dd = torch.from_numpy(D).cuda()
    for k in (1, 10, 100, 1000):
        want = E.topk_by_distance(D, k)
        for chunked in (False, True):            # one block per row / chunks + merge
            idx, val = b.emb_topk_min(Dd, k, chunked=chunked)
            assert np.array_equal(idx.cpu().numpy(), want), (k, chunked)
            assert np.array_equal(val.cpu().numpy(), np.take_along_axis(D, want, 1)), (k, chunked)
    # A last chunk shorter than k (12288-entry chunks), a single chunk, and a row whose
    # k smallest all sit in the last chunk.
    for N, k in ((2 * 12288 + 50, 100), (700, 333), (3 * 12288 + 7, 64)):
        D2 = rng.integers(0, 50, size=(4, N)).astype(np.float32)
        D2[3, -k:] = -1.0
        want = E.topk_by_distance(D2, k)
        idx, val = b.emb_topk_min(torch.from_numpy(D2).cuda(), k, chunked=True)
        assert np.array_equal(idx.cpu().numpy(), want), (N, k)
        assert np.array_equal(val.cpu().numpy(), np.take_along_axis(D2, want, 1)), (N, k)


@pytest.mark.parametrize("N", [300_000, 50_000])
def test_topk_min_long_rows_bound_and_filter(N):
    """Rows of 300,000 (bound-and-filter with 8,192-entry chunks) and 50,000 (2,048-entry
    chunks for k = 100): random distances, heavy ties, an all-equal row (its list
    overflows: one-block fallback), negatives, and the smallest entries packed in the
    last, partial chunk."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    rng = np.random.default_rng(12)
    M = 5
    D = rng.standard_normal((M, N)).astype(np.float32) * 50 + 900
    D[1] = rng.integers(0, 40, N).astype(np.float32)          # ties
    D[2] = 3.0                                                 # all equal
    D[3, ::997] = -2.0                                         # negatives spread out
    D[4, -200:] = 1.0                                          # minima in the partial chunk
    Dd = torch.from_numpy(D).cuda()
    for k in (1, 7, 100):
        want = E.topk_by_distance(D, k)
        idx, val = b.emb_topk_min(Dd, k, chunked=True)
        assert np.array_equal(idx.cpu().numpy(), want), k
        assert np.array_equal(val.cpu().numpy(), np.take_along_axis(D, want, 1)), k


def test_rerank_bit_exact_and_full_candidate_set_equals_scan():
    need_gpu()
    gen = synth.SMALL
    n, nq = 300, 6
    say("rerank: build")
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    labels[2] = 0                                                # an empty query
    rng = np.random.default_rng(8)
    cand = np.stack([rng.choice(n, 100, replace=False) for _ in range(nq)]).astype(np.int32)
    lab_d = torch.from_numpy(labels).cuda()
    idx, score, counts = db.rerank(lab_d, torch.from_numpy(cand).cuda(), 10)
    db.sync()
    for q in range(nq):
        cnt, sc = oracle.scan_block(conc[cand[q]], labels[q], synth.T_LO, synth.T_HI)
        order = sorted(range(100), key=lambda j: (-sc[j], cand[q][j]))[:10]
        assert idx[q].cpu().tolist() == [int(cand[q][j]) for j in order]
        assert np.array_equal(score[q].cpu().numpy().view(np.uint64), sc[order].view(np.uint64))
        assert np.array_equal(counts[q].cpu().numpy().view(np.uint32).astype(np.uint64), cnt[order])
    # Candidates = every entry: the rerank reproduces the exact scan bit for bit.
    allc = torch.arange(n, dtype=torch.int32).repeat(nq, 1).cuda()
    ri, rs, rc = db.rerank(lab_d, allc, 10)
    for q in range(nq):
        si, ss, sc_ = db.query(lab_d[q], 10)
        db.sync()
        assert torch.equal(ri[q], si) and torch.equal(rs[q], ss) and torch.equal(rc[q], sc_)


@pytest.mark.parametrize("nq,nc", [(70, 100), (96, 128)])
def test_rerank_batch_with_shared_candidates_bit_exact(nq, nc):
    """A batch of many queries whose candidates are drawn from 150 entries (each entry a
    candidate of many queries): the top-k, scores and counts equal the oracle's exhaustive
    loop and those of the same queries reranked in batches of 10, bit for bit; an empty query
    and a one-voxel query among them."""
    need_gpu()
    gen = synth.SMALL
    n = 300
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    labels[5] = 0
    labels[9] = 0
    labels[9, 30, 31, 32] = 3
    rng = np.random.default_rng(nq + nc)
    cand = np.stack([rng.choice(150, nc, replace=False) for _ in range(nq)]).astype(np.int32)
    lab_d = torch.from_numpy(labels).cuda()
    cand_d = torch.from_numpy(cand).cuda()
    k = 12
    idx, score, counts = db.rerank(lab_d, cand_d, k)
    db.sync()
    cnt, sc = oracle.scan_block_multi(conc[:150], labels, synth.T_LO, synth.T_HI)
    for q in range(nq):
        order = sorted(range(nc), key=lambda j: (-sc[q, cand[q][j]], cand[q][j]))[:k]
        assert idx[q].cpu().tolist() == [int(cand[q][j]) for j in order], q
        assert np.array_equal(score[q].cpu().numpy().view(np.uint64),
                              sc[q, cand[q][order]].view(np.uint64)), q
        assert np.array_equal(counts[q].cpu().numpy().view(np.uint32).astype(np.uint64),
                              cnt[q, cand[q][order]]), q
    for q0 in range(0, nq, 10):
        pi, ps, pc = db.rerank(lab_d[q0:q0 + 10], cand_d[q0:q0 + 10], k)
        db.sync()
        assert torch.equal(pi, idx[q0:q0 + 10]) and torch.equal(ps, score[q0:q0 + 10])
        assert torch.equal(pc, counts[q0:q0 + 10])


def test_query_embed_chain_matches_its_parts():
    need_gpu()
    from paper_2205_04550_amd import binding as b, nn
    gen = synth.SMALL
    n, nq = 400, 8
    db, conc = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    model = nn.AutoEncoder(grid=32, latent=64, seed=1)
    with torch.no_grad():
        xl = model.encode(nn.meanpool_db(db, torch.arange(n, dtype=torch.int32, device="cuda")))
        labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
        lab_d = torch.from_numpy(labels).cuda()
        ql = model.encode(nn.meanpool_labels(lab_d))
    for fmt in (b.EMB_BF16, b.EMB_FP8):
        X, Q = b.Latents(xl, fmt), b.Latents(ql, fmt)
        idx, score, counts, ci, cd = db.query_embed(fmt, Q, X, lab_d, 50, 10)
        db.sync()
        D = b.emb_distances(Q, X)
        ti, tv = b.emb_topk_min(D, 50)
        assert torch.equal(ci, ti)
        # The reported candidate distances are the direct form of the stored vectors.
        dq, dx = _dequant(Q), _dequant(X)
        ci_h = ci.cpu().numpy()
        d64 = np.stack([((dx[ci_h[q]] - dq[q]) ** 2).sum(axis=1) for q in range(nq)])
        assert np.all(np.abs(cd.cpu().numpy().astype(np.float64) - d64) <= 1e-5 * d64)
        ri, rs, rc = db.rerank(lab_d, ci, 10)
        assert torch.equal(idx, ri) and torch.equal(score, rs) and torch.equal(counts, rc)


def test_rerank_in_two_calls_matches_rerank():
    """db_rerank_pack on a second stream, then db_rerank_packed after an event: the same
    top-k, scores and counts as db_rerank, bit for bit (an empty query included)."""
    need_gpu()
    gen = synth.SMALL
    n, nq = 200, 7
    db, _ = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.BATCH_QUERY_SEED)
    labels[3] = 0
    lab_d = torch.from_numpy(labels).cuda()
    rng = np.random.default_rng(21)
    cand = torch.from_numpy(np.stack([rng.choice(n, 40, replace=False) for _ in range(nq)])
                            .astype(np.int32)).cuda()
    want = db.rerank(lab_d, cand, 9)
    ws = db.rerank_workspace(nq)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        db.rerank_pack(lab_d, ws)
    done = torch.cuda.Event()
    done.record(side)
    torch.cuda.current_stream().wait_event(done)
    got = db.rerank_packed(ws, cand, 9)
    db.sync()
    for a, w in zip(got, want):
        assert torch.equal(a, w)


def test_two_halves_on_two_streams_match_one_stream():
    """A batch reranked as two halves at once, each on its own stream with its own workspace
    (packing with pooled counts, then the bound-ordered rerank of 60 candidates), gives the
    one-stream top-k, scores and counts, bit for bit."""
    need_gpu()
    gen = synth.SMALL
    n, nq, nc, k = 300, 24, 60, 15
    db, _ = build_db_from_host(gen, n, synth.T_LO, synth.T_HI)
    labels, _ = synth.make_queries(gen, n, nq, synth.QUERY_SEED)
    labels[5] = 0
    lab_d = torch.from_numpy(labels).cuda()
    rng = np.random.default_rng(33)
    cand = torch.from_numpy(np.stack([rng.choice(n, nc, replace=False) for _ in range(nq)])
                            .astype(np.int32)).cuda()
    want = db.rerank(lab_d, cand, k)
    cur = torch.cuda.current_stream()
    outs = []
    for h in range(2):
        a, b = h * nq // 2, (h + 1) * nq // 2
        st = torch.cuda.Stream()
        st.wait_stream(cur)
        with torch.cuda.stream(st):
            ws = db.rerank_workspace(b - a)
            pooled = torch.empty((b - a, gen.nz // 2, gen.ny // 2, gen.nx // 2), dtype=torch.uint8,
                                 device="cuda")
            db.rerank_pack_pool(lab_d[a:b], ws, pooled)
            outs.append(db.rerank_packed(ws, cand[a:b], k))
        cur.wait_stream(st)
    db.sync()
    bits = lambda t: t.view(torch.int64) if t.dtype == torch.float64 else t
    for i in range(3):
        assert torch.equal(bits(torch.cat([o[i] for o in outs])), bits(want[i])), i


@pytest.mark.parametrize("fmt", [0, 1])
def test_latents_quantised_on_a_side_stream(fmt):
    """Quantisation enqueued on another stream (the float32 copy of the input is made on
    the current stream) gives the same codes, scales and norms as on the current stream."""
    need_gpu()
    from paper_2205_04550_amd import binding as b
    lat = _lat(300, 128, 13).cuda().to(torch.float16)      # converted to float32 inside
    want = b.Latents(lat, fmt)
    side = torch.cuda.Stream()
    got = b.Latents(lat, fmt, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(got.codes.view(torch.uint8), want.codes.view(torch.uint8))
    assert torch.equal(got.sq, want.sq)
    if fmt == b.EMB_FP8:
        assert torch.equal(got.scale, want.scale)
