"""Pins for the oracle's Code 5 with independent uniforms: the offspring law
is Multinomial(n, w/W), every particle's ancestor has law w/W independently
of the others, the search is the upper bound in exact arithmetic, and the
points lie on the 53-bit lattice of [0, n)."""
import itertools
import math
from collections import Counter
from fractions import Fraction

import numpy as np

import oracle
from lawtest import chi2_ok, frac_weights
from test_oracle_collective import exact_r, multinomial_pmf, offspring


def test_offspring_law_is_multinomial():
    w = np.array([0.3, 0.9, 0.05, 0.5])
    n = len(w)
    pmf = multinomial_pmf(w, n)
    K = 20000
    obs = Counter(offspring(oracle.multinomial_iid(w, seed=5, offset=rep)[0], n)
                  for rep in range(K))
    keys = sorted(set(pmf) | set(obs))
    ok, chi2, dof = chi2_ok([obs[k] for k in keys], [pmf.get(k, 0) for k in keys])
    assert ok, (chi2, dof)


def test_ancestors_are_independent_draws_from_w():
    """Joint law of (a_0, a_2) is the product of w/W with itself, and the
    marginal of every position is w/W."""
    w = np.array([1.0, 0.0, 2.0, 0.5, 0.25])
    n = len(w)
    fw = frac_weights(w)
    pi = [x / sum(fw) for x in fw]
    K = 20000
    A = np.array([oracle.multinomial_iid(w, seed=9, offset=rep)[0] for rep in range(K)])
    assert not np.any(A == 1)  # zero weight never chosen
    pairs = Counter(zip(A[:, 0], A[:, 2]))
    cells = list(itertools.product(range(n), repeat=2))
    ok, chi2, dof = chi2_ok([pairs[c] for c in cells], [pi[c[0]] * pi[c[1]] for c in cells])
    assert ok, (chi2, dof)
    for pos in range(n):
        counts = np.bincount(A[:, pos], minlength=n)
        ok, chi2, dof = chi2_ok(counts, pi)
        assert ok, (pos, chi2, dof)


def test_search_is_upper_bound_in_exact_arithmetic_and_points_on_the_lattice():
    g = np.random.default_rng(4)
    for trial in range(40):
        n = int(2 ** g.integers(0, 7))
        w = g.random(n) ** 2
        w[g.random(n) < 0.2] = 0
        if w.sum() == 0:
            w[0] = 1
        a, fl, r, p = oracle.multinomial_iid(w, seed=trial, return_rp=True)
        assert fl == 0
        assert np.all((p >= 0) & (p < n))
        # n a power of two: p = n u is exact, so p 2^53 / n is an integer below 2^53
        m = p * 2.0**53 / n
        assert np.all(m == np.floor(m)) and np.all(m < 2.0**53)
        R = exact_r(w)
        want = [min(sum(1 for i in range(n - 1) if R[i] <= Fraction(float(pk))), n - 1)
                for pk in p]
        assert list(a) == want


def test_degenerate_inputs():
    assert oracle.multinomial_iid(np.zeros(4))[1] == oracle.FLAG_ZERO_TOTAL
    a, fl = oracle.multinomial_iid(np.array([1.0, np.nan]))
    assert fl == oracle.FLAG_BAD_WEIGHTS and list(a) == [0, 1]
    a, fl = oracle.multinomial_iid(np.array([0.0, 0.0, 3.0]))
    assert fl == 0 and list(a) == [2, 2, 2]
    assert math.isfinite(oracle.multinomial_iid(np.ones(1), return_rp=True)[3][0])
