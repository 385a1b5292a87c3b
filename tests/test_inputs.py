"""The synthetic weight generator matches the paper's closed-form moments."""
import math

import numpy as np

from paper_1301_4019_amd import inputs


def test_weight_moments_match_closed_forms():
    n = 400000
    for y in (0.0, 1.0, 2.0, 3.0, 4.0):
        w = inputs.weights(n, y, seed=3, dtype=np.float64)
        m, m2 = inputs.expected_weight(y), inputs.expected_weight_sq(y)
        se_mean = math.sqrt((m2 - m * m) / n)
        assert abs(w.mean() - m) < 5 * se_mean
        # second moment: its standard error from E[w^4] = 5^{-1/2} exp(-2 y^2 / 5)
        m4 = 5 ** -0.5 * math.exp(-2 * y * y / 5)
        assert abs((w * w).mean() - m2) < 5 * math.sqrt((m4 - m2 * m2) / n)
        assert w.max() <= 1.0


def test_weights_are_reproducible_and_rounded_once():
    a = inputs.weights(1000, 2.0, seed=9)
    b = inputs.weights(1000, 2.0, seed=9)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    w64 = inputs.weights(1000, 2.0, seed=9, dtype=np.float64)
    assert np.array_equal(w64.astype(np.float32), a)


def test_ragged_batch_shape():
    w, off, ys = inputs.ragged_batch(n_filters=64, seed=1)
    sizes = np.diff(off)
    assert off[0] == 0 and off[-1] == w.size
    assert sizes.min() >= 2**8 and sizes.max() <= 2**16
    assert np.all((ys >= 0) & (ys <= 4))
