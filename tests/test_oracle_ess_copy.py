"""Pins for the oracle's effective sample size (section 3.4) and the copy
step of section 2.3 (out-of-place form), from closed forms, invariants and
brute force rather than the formulas themselves."""
import itertools
import math
import random

import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs


# ------------------------------------------------------------------ ESS
def test_ess_equal_weights_is_the_count():
    for n in (1, 2, 7, 1000):
        for v in (1.0, 0.3, 1e-30, 1e300):
            assert oracle.ess(np.full(n, v)) == (n, 0)


def test_ess_k_equal_weights_among_zeros_is_k():
    rng = np.random.default_rng(0)
    for n, k in ((10, 1), (10, 3), (1000, 17), (4096, 4096)):
        w = np.zeros(n)
        w[rng.choice(n, k, replace=False)] = 2.5
        assert oracle.ess(w) == (k, 0)


def test_ess_bounds_and_invariances():
    """1 <= ESS <= n (Cauchy-Schwarz), equality at n only for equal weights;
    ESS is invariant to scaling (exactly, by powers of two) and to order."""
    rng = np.random.default_rng(1)
    for n in (2, 3, 50, 999):
        w = rng.exponential(size=n)
        e, fl = oracle.ess(w)
        assert fl == 0 and 1.0 <= e < n
        assert oracle.ess(w * 2.0**-700)[0] == e
        assert oracle.ess(w * 2.0**500)[0] == e
        assert oracle.ess(w[::-1].copy())[0] == pytest.approx(e, rel=1e-15)
        assert oracle.ess(w * 3.7)[0] == pytest.approx(e, rel=1e-15)


def test_ess_two_valued_closed_form():
    """m weights a, n - m weights b: ESS = (ma + (n-m)b)^2 / (ma^2 + (n-m)b^2),
    which for b = 0 is m and for a = 2b, m = n/2 is 9n/10."""
    assert oracle.ess(np.r_[np.full(50, 2.0), np.full(50, 1.0)])[0] == pytest.approx(90.0,
                                                                                      rel=1e-15)
    assert oracle.ess(np.r_[np.full(3, 4.0), np.full(1, 0.0)])[0] == 3.0


@pytest.mark.parametrize("y", [0.0, 1.0, 2.0])
def test_ess_law_of_large_numbers(y):
    """For the paper's weight sets (log w = -(x - y)^2 / 2, x ~ N(0, 1)),
    E[w] = exp(-y^2/4) / sqrt(2) and E[w^2] = exp(-y^2/3) / sqrt(3), so
    ESS / n tends to E[w]^2 / E[w^2] = (sqrt(3) / 2) exp(-y^2 / 6)."""
    n = 1 << 20
    w = inputs.weights(n, y, seed=3).astype(np.float64)
    limit = math.sqrt(3.0) / 2.0 * math.exp(-y * y / 6.0)
    assert oracle.ess(w)[0] / n == pytest.approx(limit, rel=5e-3)


def test_ess_edge_cases():
    assert oracle.ess(np.zeros(0)) == (0.0, 0)
    assert oracle.ess(np.zeros(5)) == (0.0, oracle.FLAG_ZERO_TOTAL)
    for bad in (-1.0, np.nan, np.inf):
        e, fl = oracle.ess(np.array([1.0, bad, 1.0]))
        assert math.isnan(e) and fl == oracle.FLAG_BAD_WEIGHTS
    # squares of binary64 weights beyond 1e154 overflow binary64 but not the oracle
    assert oracle.ess(np.array([1e300, 1e300, 0.0])) == (2.0, 0)


# ------------------------------------------------------------------ copy
def in_place_copy(c, x, order):
    """The copy step run in place on one buffer, particles visited in `order`."""
    x = x.copy()
    for i in order:
        if c[i] != i:
            x[i] = x[c[i]]
    return x


def test_copy_equals_in_place_in_any_order_brute_force():
    """For every ancestry with n <= 5, the permuted ancestry of Code 10 makes
    the in-place copy independent of the visiting order, equal to the out of
    place copy, and a rearrangement of the rows x[a_i]."""
    rnd = random.Random(0)
    for n in range(1, 6):
        x = np.arange(n * 2, dtype=np.float64).reshape(n, 2) + 0.5
        for a in itertools.product(range(n), repeat=n):
            a = np.array(a, dtype=np.int32)
            c, _ = oracle.permute(a)
            out, fl = oracle.copy_rows(c, x)
            assert fl == 0
            for _ in range(3):
                order = list(range(n))
                rnd.shuffle(order)
                assert np.array_equal(in_place_copy(c, x, order), out)
            assert sorted(map(tuple, out)) == sorted(map(tuple, x[a]))


def test_copy_of_an_unpermuted_ancestry_is_flagged():
    """a = (1, 2, 2): slot 1 is both read (by 0) and written (from 2), which
    the in-place predicate forbids; particle 0 keeps its row."""
    x = np.array([[10.0], [11.0], [12.0]])
    out, fl = oracle.copy_rows(np.array([1, 2, 2]), x)
    assert fl == oracle.FLAG_BAD_ANCESTOR
    assert out[:, 0].tolist() == [10.0, 12.0, 12.0]
    out, fl = oracle.copy_rows(np.array([0, 5, -1]), x)
    assert fl == oracle.FLAG_BAD_ANCESTOR and np.array_equal(out, x)


def test_copy_identity_and_one_survivor():
    x = np.random.default_rng(2).normal(size=(6, 3))
    assert np.array_equal(oracle.copy_rows(np.arange(6), x)[0], x)
    out, fl = oracle.copy_rows(np.full(6, 4), x)
    assert fl == 0 and np.all(out == x[4])
