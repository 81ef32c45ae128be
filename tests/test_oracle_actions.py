"""Pins of the oracle's discretized actions (Sec. 5.2, Expert: discretizing
the continuous inverse): bin centres, half-way points, clamping."""
import numpy as np

import oracle


def test_bin_centres_map_to_themselves():
    lo, hi, bins = -6.0, 6.0, 13            # centres at the integers -6..6 (exact in binary32)
    v = np.arange(-6, 7, dtype=np.float32)
    idx, snp = oracle.discretize(v, lo, hi, bins)
    np.testing.assert_array_equal(idx, np.arange(13))
    np.testing.assert_array_equal(snp, v)


def test_nearest_half_up_and_clamp():
    lo, hi, bins = -1.0, 1.0, 5             # centres -1, -0.5, 0, 0.5, 1
    v = np.array([-0.26, -0.25, -0.24, 0.74, 0.75, 0.76, -3.0, 9.0, 1.0, -1.0], np.float32)
    idx, snp = oracle.discretize(v, lo, hi, bins)
    # -0.25 is half-way between -0.5 and 0 (exact in binary32): it goes up
    np.testing.assert_array_equal(idx, [1, 2, 2, 3, 4, 4, 0, 4, 4, 0])
    np.testing.assert_array_equal(snp, np.array([-0.5, 0, 0, 0.5, 1, 1, -1, 1, 1, -1], np.float32))


def test_error_is_at_most_half_a_bin():
    rng = np.random.default_rng(8)
    lo, hi, bins = -0.3, 0.3, 31
    v = rng.uniform(lo, hi, 5000).astype(np.float32)
    idx, snp = oracle.discretize(v, lo, hi, bins)
    step = (hi - lo) / (bins - 1)
    assert (np.abs(snp.astype(np.float64) - v) <= 0.5 * step + 1e-6).all()
    assert idx.min() >= 0 and idx.max() <= bins - 1
    assert (np.diff(idx[np.argsort(v, kind="stable")]) >= 0).all()   # monotone in the value
