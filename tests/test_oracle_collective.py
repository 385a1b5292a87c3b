"""Pins for the oracle's stratified (Code 7), systematic (Code 8) and
multinomial (Code 5) resamplers.

Exact laws for tiny n: stratum s (0-based) holds the point s + 1 - u_s, uniform
on (s, s+1], and picks the particle i whose interval (r_{i-1}, r_i] contains
it, so P(a_s = i) is the length of (r_{i-1}, r_i] within (s, s+1]; strata are
independent for the stratified scheme and share one offset for the systematic
one.  Multinomial offspring follow Multinomial(n, w/W).
"""
import itertools
import math
from collections import Counter
from fractions import Fraction

import numpy as np

import oracle
from lawtest import chi2_ok, frac_weights

W4 = np.array([0.5, 0.125, 0.0, 0.875])


def exact_r(w):
    fw = frac_weights(w)
    W = sum(fw)
    n = len(fw)
    r, acc = [], Fraction(0)
    for x in fw:
        acc += x
        r.append(n * acc / W)
    return r


def stratum_probs(w):
    r = exact_r(w)
    n = len(w)
    P = [[Fraction(0)] * n for _ in range(n)]
    for s in range(n):
        lo_s, hi_s = Fraction(s), Fraction(s + 1)
        prev = Fraction(0)
        for i in range(n):
            lo, hi = max(prev, lo_s), min(r[i], hi_s)
            if hi > lo:
                P[s][i] = hi - lo
            prev = r[i]
    return P


def code7_literal(w, u):
    """Code 7 as printed (1-based, exact rationals), then Code 11."""
    fw = frac_weights(w)
    n = len(fw)
    W = [sum(fw[:i + 1]) for i in range(n)]
    uu = [None] + [Fraction(x) for x in u]  # u^1..u^N
    O = []
    for i in range(1, n + 1):
        r = n * W[i - 1] / W[n - 1]
        k = min(n, math.floor(r) + 1)
        O.append(min(n, math.floor(r + uu[k])))
    a = []
    start = 0
    for i in range(1, n + 1):
        a.extend([i] * (O[i - 1] - start))
        start = O[i - 1]
    return [x - 1 for x in a]


def offspring(a, n):
    return tuple(np.bincount(a, minlength=n))


def test_stratified_matches_code7_in_exact_arithmetic():
    g = np.random.default_rng(21)
    for trial in range(60):
        n = int(g.integers(1, 40))
        w = g.random(n) ** int(g.integers(1, 6))
        w[g.random(n) < 0.2] = 0.0
        if w.sum() == 0:
            w[0] = 1.0
        if trial % 2:
            w = w.astype(np.float32).astype(np.float64)
        u = oracle.stratum_offsets(n, seed=trial, offset=3)
        a, fl = oracle.stratified_u(w, u)
        assert fl == 0
        assert list(a) == code7_literal(w, u), trial


def test_stratified_per_stratum_law():
    K = 20000
    n = len(W4)
    counts = np.zeros((n, n))
    for rep in range(K):
        a, fl = oracle.stratified(W4, seed=4, offset=rep)
        counts[np.arange(n), a] += 1
    P = stratum_probs(W4)
    for s in range(n):
        ok, chi2, dof = chi2_ok(counts[s], P[s])
        assert ok, (s, chi2, dof)


def test_stratified_joint_offspring_law():
    # strata are independent: enumerate all stratum outcomes
    w = np.array([0.3, 0.9, 0.05, 0.5])
    n = len(w)
    P = stratum_probs(w)
    pmf = Counter()
    for choice in itertools.product(range(n), repeat=n):
        p = Fraction(1)
        for s, i in enumerate(choice):
            p *= P[s][i]
        if p:
            pmf[offspring(np.array(choice), n)] += p
    K = 20000
    obs = Counter(offspring(oracle.stratified(w, seed=6, offset=rep)[0], n) for rep in range(K))
    keys = sorted(set(pmf) | set(obs))
    ok, chi2, dof = chi2_ok([obs[k] for k in keys], [pmf.get(k, 0) for k in keys])
    assert ok, (chi2, dof)


def test_systematic_offspring_floor_ceil_and_identity_with_stratified():
    g = np.random.default_rng(5)
    for trial in range(200):
        n = int(g.integers(1, 60))
        w = g.random(n) ** 3
        w[g.random(n) < 0.1] = 0.0
        if w.sum() == 0:
            w[-1] = 0.5
        a, fl = oracle.systematic(w, seed=trial)
        assert fl == 0
        o = np.bincount(a, minlength=n)
        assert o.sum() == n
        fw = frac_weights(w)
        W = sum(fw)
        for i in range(n):
            e = n * fw[i] / W
            assert math.floor(e) <= o[i] <= math.ceil(e)
        u0 = oracle.systematic_offset(seed=trial)
        a2, _ = oracle.stratified_u(w, np.full(n, u0))
        assert np.array_equal(a, a2)


def test_systematic_law_single_offset():
    # the whole ancestry is a function of one uniform offset
    w = np.array([0.3, 0.9, 0.05, 0.5])
    n = len(w)
    r = exact_r(w)
    # breakpoints of offspring(u) where some point s + 1 - u crosses an r_i
    br = sorted({Fraction(0), Fraction(1)} | {1 - (ri - math.floor(ri)) for ri in r if 0 < ri - math.floor(ri)})
    pmf = Counter()
    for lo, hi in zip(br[:-1], br[1:]):
        mid = (lo + hi) / 2
        a, _ = oracle.stratified_u(w, np.full(n, float(mid)))
        pmf[offspring(a, n)] += hi - lo
    K = 20000
    obs = Counter(offspring(oracle.systematic(w, seed=9, offset=rep)[0], n) for rep in range(K))
    keys = sorted(set(pmf) | set(obs))
    ok, chi2, dof = chi2_ok([obs[k] for k in keys], [pmf.get(k, 0) for k in keys])
    assert ok, (chi2, dof)


def test_collective_invariants_random_weights():
    g = np.random.default_rng(17)
    for trial in range(40):
        n = int(g.integers(1, 3000))
        w = np.exp(-0.5 * (g.standard_normal(n) - 3.0) ** 2).astype(np.float32)
        w[g.random(n) < 0.05] = 0
        if w.sum() == 0:
            w[0] = 1
        for fn in (oracle.stratified, oracle.systematic, oracle.multinomial):
            a, fl = fn(w, seed=trial)
            assert fl == 0
            assert a.min() >= 0 and a.max() < n
            assert np.all(np.diff(a) >= 0)            # sorted ancestry
            assert not np.any(w[a] == 0)              # zero weights never chosen
        o = np.bincount(oracle.stratified(w, seed=trial)[0], minlength=n)
        e = n * w.astype(np.float64) / w.astype(np.float64).sum()
        assert np.all(np.abs(o - e) < 2)


def multinomial_pmf(w, n):
    fw = frac_weights(w)
    W = sum(fw)
    pi = [x / W for x in fw]
    pmf = {}
    for o in itertools.product(range(n + 1), repeat=len(w)):
        if sum(o) != n:
            continue
        p = Fraction(math.factorial(n))
        for oi, pii in zip(o, pi):
            p = p / math.factorial(oi) * pii**oi
        if p:
            pmf[o] = p
    return pmf


def test_multinomial_offspring_law():
    w = np.array([0.3, 0.9, 0.05, 0.5])
    n = len(w)
    pmf = multinomial_pmf(w, n)
    K = 20000
    obs = Counter(offspring(oracle.multinomial(w, seed=12, offset=rep)[0], n) for rep in range(K))
    keys = sorted(set(pmf) | set(obs))
    ok, chi2, dof = chi2_ok([obs[k] for k in keys], [pmf.get(k, 0) for k in keys])
    assert ok, (chi2, dof)


def test_multinomial_sorted_points_are_uniform_order_statistics():
    n = 5
    K = 20000
    ps = np.array([oracle.multinomial(np.ones(n), seed=1, offset=rep, return_rp=True)[3]
                   for rep in range(K)])
    assert np.all(np.diff(ps, axis=1) >= 0) and ps.min() >= 0 and ps.max() < n
    # p_k / n ~ Beta(k+1, n-k): mean (k+1)/(n+1), var (k+1)(n-k)/((n+1)^2 (n+2))
    for k in range(n):
        m = (k + 1) / (n + 1)
        v = (k + 1) * (n - k) / ((n + 1) ** 2 * (n + 2))
        assert abs(ps[:, k].mean() / n - m) < 6 * math.sqrt(v / K)
        assert abs(ps[:, k].var() / n**2 - v) < 0.1 * v


def test_multinomial_search_is_upper_bound_in_exact_arithmetic():
    g = np.random.default_rng(2)
    for trial in range(50):
        n = int(g.integers(1, 50))
        w = g.random(n) ** 2
        w[g.random(n) < 0.2] = 0
        if w.sum() == 0:
            w[0] = 1
        r = exact_r(w)
        p = np.sort(g.random(n) * n)
        # include exact boundary hits: a point equal to r_i goes to particle i+1
        if n > 2:
            p[0] = float(r[0]) if Fraction(float(r[0])) == r[0] else p[0]
            p = np.sort(p)
        a, fl = oracle.multinomial_points(w, p)
        want = [min(sum(1 for i in range(n - 1) if r[i] <= Fraction(float(pk))), n - 1) for pk in p]
        assert list(a) == want


def code6_serial(w, g):
    """The paper's Code 6 (serial single-pass multinomial) with numpy uniforms."""
    n = len(w)
    Wex = np.concatenate([[0.0], np.cumsum(w)[:-1]])  # exclusive prefix, 1-based W^1..W^N
    total = Wex[-1] + w[-1]
    ln_max = 0.0
    j = n  # 1-based
    a = np.zeros(n, dtype=np.int64)
    for i in range(n, 0, -1):
        u = g.random()
        ln_max += math.log(u) / i
        uu = total * math.exp(ln_max)
        while uu < Wex[j - 1]:
            j -= 1
        a[i - 1] = j - 1
    return a


def test_code6_serial_multinomial_has_the_same_law():
    w = np.array([0.3, 0.9, 0.05, 0.5])
    n = len(w)
    pmf = multinomial_pmf(w, n)
    g = np.random.default_rng(77)
    K = 20000
    obs = Counter(offspring(code6_serial(w, g), n) for _ in range(K))
    keys = sorted(set(pmf) | set(obs))
    ok, chi2, dof = chi2_ok([obs[k] for k in keys], [pmf.get(k, 0) for k in keys])
    assert ok, (chi2, dof)


def test_degenerate_inputs():
    for fn in (oracle.stratified, oracle.systematic, oracle.multinomial):
        a, fl = fn(np.zeros(8))
        assert fl & oracle.FLAG_ZERO_TOTAL and np.array_equal(a, np.arange(8))
        a, fl = fn(np.array([1.0, np.nan, 2.0]))
        assert fl & oracle.FLAG_BAD_WEIGHTS and np.array_equal(a, np.arange(3))
        a, fl = fn(np.array([1.0, -1.0, 2.0]))
        assert fl & oracle.FLAG_BAD_WEIGHTS
        a, fl = fn(np.array([1.0, np.inf]))
        assert fl & oracle.FLAG_BAD_WEIGHTS
        a, fl = fn(np.array([3.5]))
        assert fl == 0 and list(a) == [0]
        a, fl = fn(np.array([0.0, 0.0, 5.0, 0.0]))
        assert fl == 0 and list(a) == [2, 2, 2, 2]
