"""Seeded input generator: determinism and the shape of what it makes."""
import hashlib

import numpy as np

import oracle
import synth


def test_same_bytes_for_any_thread_count():
    a = synth.SMALL.conc_cpu(10, 5, threads=1)
    b = synth.SMALL.conc_cpu(10, 5, threads=7)
    assert hashlib.sha256(a.tobytes()).digest() == hashlib.sha256(b.tobytes()).digest()
    # Chunking does not matter either: entry 12 alone equals entry 12 of the block.
    c = synth.SMALL.conc_cpu(12, 1, threads=3)
    assert np.array_equal(c[0], a[2])


def test_values_in_unit_interval_and_zero_outside_brain():
    c = synth.SMALL.conc_cpu(0, 8)
    assert c.min() >= 0.0 and c.max() <= 1.0
    assert not np.isnan(c).any()
    nz, ny, nx = c.shape[1:]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = ((x - (nx - 1) / 2) / (0.40 * nx)) ** 2 + ((y - (ny - 1) / 2) / (0.46 * ny)) ** 2 + \
          ((z - (nz - 1) / 2) / (0.36 * nz)) ** 2 > 1.0 + 1e-9
    assert np.all(c[:, out] == 0.0)
    # No float32 denormals are written (values below 2^-126 are exactly 0).
    nz_vals = c[c != 0]
    assert nz_vals.min() >= np.finfo(np.float32).tiny


def test_logistic_matches_libm_to_float_rounding():
    """The generator's own exp agrees with libm's exp after rounding to float32."""
    gen = synth.SMALL
    p = gen.params(0, 4)
    c = gen.conc_cpu(0, 4)
    nz, ny, nx = c.shape[1:]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inside = ((x - (nx - 1) / 2) * (1 / (0.40 * nx))) ** 2 + ((y - (ny - 1) / 2) * (1 / (0.46 * ny))) ** 2 \
        + ((z - (nz - 1) / 2) * (1 / (0.36 * nz))) ** 2 <= 1.0
    for i in range(4):
        dx = (x - p[i]["cx"]) * p[i]["iax"]
        dy = (y - p[i]["cy"]) * p[i]["iay"]
        dz = (z - p[i]["cz"]) * p[i]["iaz"]
        r = np.sqrt((dx * dx + dy * dy) + dz * dz)
        t = (r - p[i]["R"]) * p[i]["iw"]
        ref = np.where(t > 80, 0.0, 1.0 / (1.0 + np.exp(np.minimum(t, 80.0)))).astype(np.float32)
        ref = np.where(inside, ref, np.float32(0))
        diff = np.abs(ref.astype(np.float64) - c[i].astype(np.float64))
        ulp = np.spacing(np.maximum(np.abs(ref), np.float32(1e-30)).astype(np.float32))
        assert np.all(diff <= ulp)


def test_parameter_ranges():
    p = synth.FULL.params(0, 2000)
    assert p["R"].min() >= 8 and p["R"].max() <= 40
    w = 1 / p["iw"]
    assert w.min() >= 1 - 1e-12 and w.max() <= 8 + 1e-12
    for a in ("iax", "iay", "iaz"):
        aa = 1 / p[a]
        assert aa.min() >= 0.7 - 1e-12 and aa.max() <= 1.3 + 1e-12
    # Centres inside the brain ellipsoid.
    g = 128
    u = ((p["cx"] - (g - 1) / 2) / (0.40 * g)) ** 2 + ((p["cy"] - (g - 1) / 2) / (0.46 * g)) ** 2 \
        + ((p["cz"] - (g - 1) / 2) / (0.36 * g)) ** 2
    assert u.max() <= 1.0 + 1e-9


def test_query_noise_flips_two_percent_of_boundary():
    gen = synth.SMALL
    src = 3
    clean = oracle.threshold(gen.conc_cpu(src, 1)[0], synth.T_LO, synth.T_HI)
    q = gen.query(src, synth.T_LO, synth.T_HI, synth.QUERY_SEED, 0)
    for bit in (1, 2):
        m = (clean & bit) != 0
        # Boundary: voxels with an in-grid 6-neighbour of the other value.
        b = np.zeros_like(m)
        for ax in range(3):
            d = np.diff(m.astype(np.int8), axis=ax) != 0
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[ax] = slice(0, -1)
            sl_hi[ax] = slice(1, None)
            b[tuple(sl_lo)] |= d
            b[tuple(sl_hi)] |= d
        flipped = ((q & bit) != 0) != m
        assert not np.any(flipped & ~b)
        assert int(flipped.sum()) == int(np.floor(0.02 * b.sum() + 0.5))
    # Deterministic.
    q2 = gen.query(src, synth.T_LO, synth.T_HI, synth.QUERY_SEED, 0)
    assert np.array_equal(q, q2)


def test_rois_inside_grid_with_side_range():
    labs, _ = synth.make_queries(synth.SMALL, 100, 6, synth.BATCH_QUERY_SEED)
    rois = synth.make_rois(labs, synth.ROI_SEED)
    for r in rois:
        for d in range(3):
            assert 0 <= r[d] < r[d + 3] <= 64
            assert 24 <= r[d + 3] - r[d] <= 64
