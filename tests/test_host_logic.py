"""Host-side checks of integer tricks the kernels rely on (run on the CPU)."""
import numpy as np


def test_reciprocal_division_is_exact_in_the_guaranteed_range():
    # Row r of a box is split as r = zr * d + yr with zr = floor(r * ceil(2^32/d) / 2^32);
    # the library guarantees r * d < 2^32 (ny * ny * nz < 2^32), d >= 2.
    for d in list(range(2, 300)) + [511, 512, 1000, 2047, 4095]:
        M = (2 ** 32 + d - 1) // d
        assert M < 2 ** 32
        rmax = (2 ** 32 - 1) // d
        r = np.unique(np.concatenate([np.arange(0, min(rmax, 200000), dtype=np.uint64),
                                      np.array([rmax - i for i in range(min(rmax, 64))], np.uint64)]))
        got = (r * np.uint64(M)) >> np.uint64(32)
        assert np.array_equal(got, r // np.uint64(d)), d
