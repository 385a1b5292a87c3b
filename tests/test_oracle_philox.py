"""Pins for the oracle's Philox4x32-10 and canonical draws."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from philox_np import philox4x32

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        ctr, key, out = (part.split() for part in line.split("|"))
        rows.append(([int(x, 16) for x in ctr], [int(x, 16) for x in key],
                     [int(x, 16) for x in out]))
    return rows


def test_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(oracle.philox4x32_10(ctr, key)) == out
        assert list(philox4x32([ctr], [key])[0]) == out


def test_matches_independent_numpy_philox():
    g = np.random.default_rng(1234)
    ctr = g.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    ref = philox4x32(ctr, key)
    for i in range(ctr.shape[0]):
        assert np.array_equal(oracle.philox4x32_10(ctr[i], key[i]), ref[i])


def test_draw_counter_layout():
    # (index, domain<<28 | step, filter, offset), key = (seed lo, seed hi)
    seed = 0x0123456789ABCDEF
    got = oracle.draw(seed, 77, 2, 5, filt=9, offset=3)
    want = philox4x32([[77, (2 << 28) | 5, 9, 3]], [[0x89ABCDEF, 0x01234567]])[0]
    assert np.array_equal(got, want)


def test_u_accept_lattice():
    assert oracle.u_accept(0) == 2.0**-32
    assert oracle.u_accept(2**32 - 1) == 1.0
    for x in [1, 12345, 2**31, 2**32 - 2]:
        assert Fraction(oracle.u_accept(x)) == Fraction(x + 1, 2**32)


def test_index_is_high_word_of_product_and_uniform():
    g = np.random.default_rng(7)
    for n in [1, 2, 3, 5, 1000, 2**20, 2**31 - 1]:
        for _ in range(50):
            x0, x1 = (int(v) for v in g.integers(0, 2**32, size=2))
            j = oracle.index(x0, x1, n)
            assert 0 <= j < n
            assert j == (((x1 << 32) | x0) * n) >> 64
    # uniformity over a small n from Philox words
    n = 7
    words = philox4x32(np.column_stack([np.arange(70000), np.zeros((70000, 3))]).astype(np.uint32),
                       np.zeros((70000, 2), dtype=np.uint32))
    counts = np.bincount([oracle.index(int(a), int(b), n) for a, b in words[:, :2]], minlength=n)
    expected = 70000 / n
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 40  # 6 dof; p ~ 1e-6


def test_accept_is_exact():
    g = np.random.default_rng(99)
    cases = []
    for _ in range(3000):
        x = int(g.integers(0, 2**32))
        u = oracle.u_accept(x)
        wk = float(g.random()) * 2.0 ** int(g.integers(-30, 30))
        if g.random() < 0.3:
            wk = float(np.float32(wk))
        # w_j near the product to exercise the boundary
        prod = Fraction(u) * Fraction(wk)
        wj = float(prod)
        for delta in (-1, 0, 1):
            wj2 = float(np.nextafter(wj, np.inf if delta > 0 else -np.inf)) if delta else wj
            cases.append((u, wk, wj2))
    for u, wk, wj in cases:
        assert oracle.accept(u, wk, wj) == (Fraction(u) * Fraction(wk) <= Fraction(wj))
    assert oracle.accept(1.0, 0.0, 0.0)
    assert not oracle.accept(2.0**-32, 1.0, 0.0)


def test_round_count_variants_match_the_numpy_implementation():
    """The round-count study's generator: the oracle's r-round Philox equals
    the independent numpy one for several round counts, and r = 10 is the
    pinned Philox4x32-10."""
    import philox_np
    g = np.random.default_rng(11)
    ctr = g.integers(0, 2**32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2**32, size=(64, 2), dtype=np.uint64).astype(np.uint32)
    for rounds in (1, 7, 10, 12):
        ref = philox_np.philox4x32(ctr, key, rounds=rounds)
        got = np.array([oracle.philox4x32_r(c, k, rounds) for c, k in zip(ctr, key)])
        assert np.array_equal(got, ref), rounds
    assert np.array_equal(oracle.philox4x32_r(ctr[0], key[0], 10),
                          oracle.philox4x32_10(ctr[0], key[0]))


def test_round_count_setting_is_scoped():
    w = np.random.default_rng(1).random(50)
    a10 = oracle.metropolis(w, 8, seed=3)
    with oracle.philox_rounds(7):
        a7 = oracle.metropolis(w, 8, seed=3)
        x7 = oracle.draw(3, 5, 2, 0)
    assert not np.array_equal(a7, a10)
    assert np.array_equal(oracle.metropolis(w, 8, seed=3), a10)
    import philox_np
    ref = philox_np.philox4x32(np.array([[5, 2 << 28, 0, 0]]), np.array([[3, 0]]), rounds=7)[0]
    assert np.array_equal(x7, ref)
    with pytest.raises(ValueError):
        with oracle.philox_rounds(0):
            pass
