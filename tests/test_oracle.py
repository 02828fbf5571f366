"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties one part of the oracle (threshold, counts, Dice, score, rank)
to something fixed by the paper's definitions (Sec. 2.3: thresholds give the
FLAIR/T1Gd masks, Dice is the metric, the two Dice values are added and the
highest sum wins, the exhaustive loop is the ground truth) or by mathematics:
hand-counted cases, closed forms for boxes and logistic fronts, identities,
exact rational arithmetic, and brute force on tiny inputs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def box_labels(shape, fl_box=None, t1_box=None):
    """uint8 [nz][ny][nx] with FLAIR / T1Gd bits set inside half-open boxes (x0,y0,z0,x1,y1,z1)."""
    lab = np.zeros(shape, dtype=np.uint8)
    for bit, b in ((1, fl_box), (2, t1_box)):
        if b is not None:
            x0, y0, z0, x1, y1, z1 = b
            lab[z0:z1, y0:y1, x0:x1] |= bit
    return lab


# --- hand-counted cases on a 32 x 2 x 2 grid --------------------------------------------

def test_hand_counted_partial_overlap():
    shape = (2, 2, 32)  # nz, ny, nx
    q = box_labels(shape, fl_box=(0, 0, 0, 8, 1, 1), t1_box=(0, 0, 0, 2, 1, 1))
    d = box_labels(shape, fl_box=(4, 0, 0, 12, 1, 1), t1_box=(10, 0, 0, 12, 1, 1))
    I_fl, I_t1, A_fl, A_t1, B_fl, B_t1 = oracle.counts(q, d)
    # FLAIR: x in [0,8) vs [4,12) share x = 4..7 -> 4 voxels; T1Gd: [0,2) vs [10,12) share none.
    assert (I_fl, A_fl, B_fl) == (4, 8, 8)
    assert (I_t1, A_t1, B_t1) == (0, 2, 2)
    assert oracle.dice(I_fl, A_fl, B_fl) == 0.5
    assert oracle.dice(I_t1, A_t1, B_t1) == 0.0
    assert oracle.score((I_fl, I_t1, A_fl, A_t1, B_fl, B_t1)) == 0.5


def test_hand_counted_whole_grid_vs_row():
    shape = (2, 2, 32)
    q = box_labels(shape, fl_box=(0, 0, 0, 32, 2, 2))          # all 128 voxels
    d = box_labels(shape, fl_box=(0, 1, 1, 32, 2, 2))          # one x-row of 32
    c = oracle.counts(q, d)
    assert c == (32, 0, 128, 0, 32, 0)
    assert oracle.dice(32, 128, 32) == 0.4
    # T1Gd masks are both empty: Dice(empty, empty) = 1, so the sum is 1.4.
    assert oracle.score(c) == 0.4 + 1.0


def test_mask_bits_are_not_swapped():
    # Query has only FLAIR; entry has only T1Gd at the same voxels: no overlap in either mask.
    shape = (2, 2, 32)
    q = box_labels(shape, fl_box=(0, 0, 0, 16, 2, 2))
    d = box_labels(shape, t1_box=(0, 0, 0, 16, 2, 2))
    assert oracle.counts(q, d) == (0, 0, 64, 0, 0, 64)
    assert oracle.score(oracle.counts(q, d)) == 0.0


# --- closed forms and identities on random boxes -----------------------------------------

def _rand_box(rng, dims):
    lo = [int(rng.integers(0, d)) for d in dims]
    hi = [int(rng.integers(l + 1, d + 1)) for l, d in zip(lo, dims)]
    return (*lo, *hi)


@pytest.mark.parametrize("seed", range(12))
def test_box_box_closed_form(seed):
    rng = np.random.default_rng(seed)
    dims = (32 * int(rng.integers(1, 3)), int(rng.integers(2, 9)), int(rng.integers(2, 9)))
    shape = dims[::-1]
    qa, qb, da, db = (_rand_box(rng, dims) for _ in range(4))
    q = box_labels(shape, qa, qb)
    d = box_labels(shape, da, db)
    roi = _rand_box(rng, dims) if seed % 2 else None
    got = oracle.counts(q, d, roi)
    R = roi or (0, 0, 0, *dims)

    def vol(*boxes):
        # |b1 n b2 n ...| of axis-aligned boxes = product over axes of the 1-D overlaps.
        return math.prod(max(0, min(b[i + 3] for b in boxes) - max(b[i] for b in boxes))
                         for i in range(3))

    assert got == (vol(qa, da, R), vol(qb, db, R), vol(qa, R), vol(qb, R), vol(da, R), vol(db, R))


@pytest.mark.parametrize("seed", range(8))
def test_count_identities(seed):
    rng = np.random.default_rng(100 + seed)
    shape = (3, 4, 64)
    q = rng.integers(0, 4, size=shape, dtype=np.uint8)
    d = rng.integers(0, 4, size=shape, dtype=np.uint8)
    I_fl, I_t1, A_fl, A_t1, B_fl, B_t1 = oracle.counts(q, d)
    assert I_fl <= min(A_fl, B_fl) and I_t1 <= min(A_t1, B_t1)
    # I(A, B) + I(A, not B) = |A|, per mask.
    c2 = oracle.counts(q, d ^ 3)
    assert I_fl + c2[0] == A_fl and I_t1 + c2[1] == A_t1
    # Symmetry of the intersection; A and B swap roles.
    r = oracle.counts(d, q)
    assert (r[0], r[1], r[2], r[3], r[4], r[5]) == (I_fl, I_t1, B_fl, B_t1, A_fl, A_t1)
    # Additivity over an ROI split into two disjoint boxes along z and along x.
    full = oracle.counts(q, d, (0, 0, 0, 64, 4, 3))
    assert full == (I_fl, I_t1, A_fl, A_t1, B_fl, B_t1)
    za = oracle.counts(q, d, (0, 0, 0, 64, 4, 1))
    zb = oracle.counts(q, d, (0, 0, 1, 64, 4, 3))
    assert tuple(a + b for a, b in zip(za, zb)) == full
    xa = oracle.counts(q, d, (0, 0, 0, 37, 4, 3))
    xb = oracle.counts(q, d, (37, 0, 0, 64, 4, 3))
    assert tuple(a + b for a, b in zip(xa, xb)) == full
    # Single-voxel ROI equals the bits of that voxel.
    v = (5, 2, 1)
    one = oracle.counts(q, d, (v[0], v[1], v[2], v[0] + 1, v[1] + 1, v[2] + 1))
    a, b = int(q[v[2], v[1], v[0]]), int(d[v[2], v[1], v[0]])
    assert one == ((a & b) & 1, (a & b) >> 1, a & 1, a >> 1, b & 1, b >> 1)


# --- Dice and score -----------------------------------------------------------------------

def test_dice_exact_rational():
    rng = np.random.default_rng(7)
    for _ in range(3000):
        A = int(rng.integers(0, 1 << 22))
        B = int(rng.integers(0, 1 << 22))
        I = int(rng.integers(0, min(A, B) + 1))
        expect = 1.0 if A + B == 0 else float(Fraction(2 * I, A + B))
        assert oracle.dice(I, A, B) == expect
        assert oracle.dice(I, B, A) == expect


def test_dice_special_cases():
    assert oracle.dice(0, 0, 0) == 1.0            # Dice(empty, empty) = 1 (reading)
    assert oracle.dice(7, 7, 7) == 1.0            # Dice(A, A) = 1
    assert oracle.dice(0, 5, 9) == 0.0            # disjoint non-empty
    assert oracle.dice(0, 5, 0) == 0.0            # one side empty


def test_score_is_sum_of_two_dice_and_bounded():
    rng = np.random.default_rng(3)
    for _ in range(500):
        A = rng.integers(0, 5000, size=2)
        B = rng.integers(0, 5000, size=2)
        I = [int(rng.integers(0, min(a, b) + 1)) for a, b in zip(A, B)]
        cnt = (I[0], I[1], int(A[0]), int(A[1]), int(B[0]), int(B[1]))
        d = [1.0 if A[m] + B[m] == 0 else float(Fraction(2 * I[m], int(A[m] + B[m])))
             for m in range(2)]
        s = oracle.score(cnt)
        assert s == d[1] + d[0]
        assert 0.0 <= s <= 2.0


def test_self_match_scores_two():
    rng = np.random.default_rng(11)
    q = rng.integers(0, 4, size=(2, 3, 32), dtype=np.uint8)
    assert oracle.score(oracle.counts(q, q)) == 2.0
    empty = np.zeros_like(q)
    assert oracle.score(oracle.counts(empty, empty)) == 2.0


# --- threshold -----------------------------------------------------------------------------

@pytest.mark.parametrize("t_lo,t_hi", [(synth.T_LO, synth.T_HI), (synth.PAPER_T_LO, synth.PAPER_T_HI)])
def test_threshold_boundary_values(t_lo, t_hi):
    f32 = np.float32
    tl, th = f32(t_lo), f32(t_hi)
    vals = np.array([0.0, np.nextafter(tl, f32(0)), tl, np.nextafter(tl, f32(1)),
                     np.nextafter(th, f32(0)), th, np.nextafter(th, f32(1)), 1.0], dtype=np.float32)
    lab = oracle.threshold(vals, t_lo, t_hi)
    # c >= t belongs to the mask: lower threshold -> bit0 (FLAIR), higher -> bit1 (T1Gd).
    assert list(lab) == [0, 0, 1, 1, 1, 3, 3, 3]


def test_threshold_float32_semantics():
    # 0.675 as float32 is 0.675000011920929; a float just below it is outside T1Gd,
    # and comparing in double against 0.675 would give the same answers (>= is robust).
    c = np.array([0.675, 0.6749999], dtype=np.float32)
    lab = oracle.threshold(c, 0.25, 0.675)
    assert list(lab) == [3, 1]
    assert list(lab >> 1) == [int(float(x) >= 0.675) for x in c]


def _r_aniso(p, shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx = (x - p["cx"]) * p["iax"]
    dy = (y - p["cy"]) * p["iay"]
    dz = (z - p["cz"]) * p["iaz"]
    return np.sqrt(dx * dx + dy * dy + dz * dz)


def _brain(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ux = (x - (nx - 1) / 2) / (0.40 * nx)
    uy = (y - (ny - 1) / 2) / (0.46 * ny)
    uz = (z - (nz - 1) / 2) / (0.36 * nz)
    return ux * ux + uy * uy + uz * uz <= 1.0


@pytest.mark.parametrize("t_lo,t_hi", [(synth.T_LO, synth.T_HI), (synth.PAPER_T_LO, synth.PAPER_T_HI)])
def test_threshold_of_logistic_front_is_ellipsoid(t_lo, t_hi):
    """1/(1+exp((r-R)/w)) >= t  <=>  r <= R + w ln((1-t)/t): each mask is an ellipsoid n brain."""
    gen = synth.SMALL
    n = 24
    conc = gen.conc_cpu(0, n)
    par = gen.params(0, n)
    shape = conc.shape[1:]
    brain = _brain(shape)
    checked = 0
    for i in range(n):
        lab = oracle.threshold(conc[i], t_lo, t_hi)
        r = _r_aniso(par[i], shape)
        w = 1.0 / par[i]["iw"]
        for bit, t in ((1, t_lo), (2, t_hi)):
            rt = par[i]["R"] + w * math.log((1 - t) / t)
            inside = (r <= rt) & brain
            far = np.abs(r - rt) > 1e-6 * np.maximum(1.0, r)
            got = (lab & bit) != 0
            assert np.array_equal(got[far], inside[far])
            checked += int(far.sum())
        # T1Gd (higher threshold) nests in FLAIR on database masks.
        assert not np.any((lab & 2) & ~((lab & 1) << 1))
    assert checked > 0.99 * 2 * n * conc[0].size


# --- ranking -------------------------------------------------------------------------------

def test_rank_matches_pairwise_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        # Few distinct values so that ties are frequent.
        sc = rng.choice([0.0, 0.5, 1.0, 1.25, 2.0], size=n)
        k = int(rng.integers(1, n + 1))
        top = oracle.rank(sc, k)
        for pos, i in enumerate(top):
            beaten_by = sum(1 for j in range(n) if sc[j] > sc[i] or (sc[j] == sc[i] and j < i))
            assert beaten_by == pos


def test_scan_duplicates_and_self_retrieval():
    """An unmodified database entry as query scores exactly 2 and the lowest duplicate wins."""
    gen = synth.SMALL
    conc = gen.conc_cpu(0, 6)
    conc = np.concatenate([conc, conc[2:3], conc[2:3]])  # entries 6 and 7 duplicate entry 2
    q = oracle.threshold(conc[2], synth.T_LO, synth.T_HI)
    cnt, sc = oracle.scan_block(conc, q, synth.T_LO, synth.T_HI)
    assert sc[2] == sc[6] == sc[7] == 2.0
    top = oracle.rank(sc, 3)
    assert top == [2, 6, 7]
    for i in range(len(sc)):
        lab = oracle.threshold(conc[i], synth.T_LO, synth.T_HI)
        assert tuple(int(v) for v in cnt[i]) == oracle.counts(q, lab)


def test_scan_block_multi_box_closed_form_and_per_query_loop():
    """The several-query loop gives, per query and box, the closed-form box overlaps and the
    same counts as thresholding each entry and counting it on its own."""
    rng = np.random.default_rng(11)
    shape = (6, 5, 64)                                  # nz, ny, nx
    n = 7
    conc = np.zeros((n,) + shape, dtype=np.float32)
    boxes = []
    for i in range(n):
        lo = [int(rng.integers(0, d - 1)) for d in (64, 5, 6)]
        hi = [int(rng.integers(l + 1, d + 1)) for l, d in zip(lo, (64, 5, 6))]
        boxes.append((lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]))
        conc[i, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = 0.9   # in both masks
    qboxes = [(3, 0, 1, 40, 4, 6), (0, 0, 0, 64, 5, 6), (31, 2, 2, 33, 3, 3)]
    queries = np.stack([box_labels(shape, b, b) for b in qboxes])
    rois = np.array([(0, 0, 0, 64, 5, 6), (10, 1, 0, 50, 5, 4), (30, 2, 2, 34, 3, 3)], np.int32)

    def inter(a, b):
        return math.prod(max(0, min(a[d + 3], b[d + 3]) - max(a[d], b[d])) for d in range(3))

    for use_roi in (False, True):
        cnt, sc = oracle.scan_block_multi(conc, queries, synth.T_LO, synth.T_HI,
                                          rois=rois if use_roi else None, threads=3)
        for j, qb in enumerate(qboxes):
            R = tuple(rois[j]) if use_roi else (0, 0, 0, 64, 5, 6)
            a = inter(qb, R)
            for i in range(n):
                b = inter(boxes[i], R)
                I = math.prod(max(0, min(qb[d + 3], boxes[i][d + 3], R[d + 3])
                                     - max(qb[d], boxes[i][d], R[d])) for d in range(3))
                assert tuple(int(v) for v in cnt[j, i]) == (I, I, a, a, b, b)
                lab = oracle.threshold(conc[i], synth.T_LO, synth.T_HI)
                assert tuple(int(v) for v in cnt[j, i]) == oracle.counts(
                    queries[j], lab, roi=R if use_roi else None)
                assert sc[j, i] == oracle.score(cnt[j, i])


def test_noisy_self_query_usually_finds_source():
    gen = synth.SMALL
    n_db = 64
    hits = 0
    for qid in range(4):
        src = synth.query_source(n_db, synth.QUERY_SEED, qid)
        q = gen.query(src, synth.T_LO, synth.T_HI, synth.QUERY_SEED, qid)
        idx, sc, cnt = oracle.query(gen, n_db, q, 3, synth.T_LO, synth.T_HI)
        hits += int(idx[0] == src)
        assert sc[0] > 1.5
    assert hits >= 3


# --- order-0 resampling (DS64 / DS32) ------------------------------------------------------

def test_resample_nearest_pins():
    # Identity when the shape is unchanged.
    rng = np.random.default_rng(2)
    lab = rng.integers(0, 4, size=(2, 6, 5, 64), dtype=np.uint8)
    assert np.array_equal(oracle.resample_nearest(lab, (6, 5, 64)), lab)
    # Samples spread evenly from the first to the last voxel: output o reads the voxel
    # nearest to o (n_in - 1) / (n_out - 1); on a ramp the output is that index.
    for n_in, n_out in ((128, 64), (128, 32), (64, 32), (37, 11)):
        ramp = np.broadcast_to(np.arange(n_in, dtype=np.int64)[:, None, None], (n_in, 2, 2)).copy()
        got = oracle.resample_nearest(ramp, (n_out, 2, 2))[:, 0, 0]
        want = [int(np.floor(o * (n_in - 1) / (n_out - 1) + 0.5)) for o in range(n_out)]
        assert got.tolist() == want
        assert got[0] == 0 and got[-1] == n_in - 1
    # Order 0 only copies values: thresholding before or after resampling is the same.
    c = synth.SMALL.conc_cpu(0, 2)
    a = oracle.resample_nearest(oracle.threshold(c, synth.T_LO, synth.T_HI), (32, 32, 32))
    b = oracle.threshold(oracle.resample_nearest(c, (32, 32, 32)), synth.T_LO, synth.T_HI)
    assert np.array_equal(a, b)


def test_moments_rowbox_com_pins():
    """Moments, row boxes and centre-of-mass keys against closed forms and brute force."""
    nz, ny, nx = 6, 5, 64
    lab = np.zeros((nz, ny, nx), np.uint8)
    assert oracle.moments(lab) == (0, 0, 0, 0)
    assert oracle.rowbox(lab) == (0, 0, 0, 0)
    lab[4, 2, 37] = 1
    assert oracle.moments(lab) == (37, 2, 4, 1)
    assert oracle.rowbox(lab) == (4, 5, 2, 3)
    # A T1Gd-only voxel widens the row box but is not part of the FLAIR moments.
    lab[1, 0, 3] = 2
    assert oracle.moments(lab) == (37, 2, 4, 1)
    assert oracle.rowbox(lab) == (1, 5, 0, 3)
    # Box [x0,x1) x [y0,y1) x [z0,z1): sum x = (area of the other two sides) * sum_{x0}^{x1-1} x.
    box = np.zeros((nz, ny, nx), np.uint8)
    x0, x1, y0, y1, z0, z1 = 5, 40, 1, 4, 2, 6
    box[z0:z1, y0:y1, x0:x1] = 3
    nxb, nyb, nzb = x1 - x0, y1 - y0, z1 - z0
    sx = nyb * nzb * (x0 + x1 - 1) * nxb // 2
    sy = nxb * nzb * (y0 + y1 - 1) * nyb // 2
    sz = nxb * nyb * (z0 + z1 - 1) * nzb // 2
    assert oracle.moments(box) == (sx, sy, sz, nxb * nyb * nzb)
    assert oracle.rowbox(box) == (z0, z1, y0, y1)
    # Brute-force loop over every voxel.
    rng = np.random.default_rng(5)
    r = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8) * rng.integers(1, 4, (nz, ny, nx),
                                                                          dtype=np.uint8)
    bx = by = bz = bc = 0
    rows = set()
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if r[z, y, x] & 1:
                    bx, by, bz, bc = bx + x, by + y, bz + z, bc + 1
                if r[z, y, x] & 3:
                    rows.add((z, y))
    assert oracle.moments(r) == (bx, by, bz, bc)
    zs = [a for a, _ in rows]
    ys = [b for _, b in rows]
    assert oracle.rowbox(r) == (min(zs), max(zs) + 1, min(ys), max(ys) + 1)
    # Keys: a 3-4-5 triangle; empty masks rank last.
    assert oracle.com_key((3, 4, 0, 1), (0, 0, 0, 1)) == np.float32(25.0)
    assert oracle.com_key((0, 0, 0, 0), (1, 1, 1, 1)) == np.float32(np.inf)
    assert oracle.com_key((2, 2, 2, 2), (1, 1, 1, 1)) == 0.0


def test_query_com_all_candidates_is_the_exact_query():
    """With every entry a candidate the prefilter changes nothing: the exact top-k."""
    rng = np.random.default_rng(11)
    n, shape = 30, (4, 6, 32)
    labs = np.stack([(rng.random(shape) < p).astype(np.uint8) * 1 +
                     (rng.random(shape) < p / 3).astype(np.uint8) * 2
                     for p in rng.uniform(0.02, 0.3, n)])
    labs[7] = labs[3]              # an exact duplicate: the lower index must win
    q = labs[3].copy()
    cand, keys, top, sc, cnt = oracle.query_com(q, labs, n, 5)
    exact = [oracle.score(oracle.counts(q, labs[i])) for i in range(n)]
    assert list(top) == oracle.rank(exact, 5)
    assert top[0] == 3 and sc[0] == 2.0
    assert sorted(cand.tolist()) == list(range(n))
    assert np.all(np.diff(keys) >= 0)
    # Candidates are the n_cand smallest keys, ties by index.
    cand4, keys4, *_ = oracle.query_com(q, labs, 4, 2)
    assert list(cand4[:2]) == [3, 7] and keys4[0] == keys4[1] == 0.0
