"""Pins for the oracle's auxiliaries: Code 11 / Code 12 conversions and the
Code 10 permutation (brute force over every ancestry vector for n <= 5)."""
import itertools
import random

import numpy as np

import oracle


def compositions(n, parts):
    if parts == 1:
        yield (n,)
        return
    for k in range(n + 1):
        for rest in compositions(n - k, parts - 1):
            yield (k,) + rest


def test_offspring_ancestor_round_trips():
    for n in range(1, 7):
        for o in compositions(n, n):
            a, fl = oracle.offspring_to_ancestors(np.array(o))
            assert fl == 0
            assert np.all(np.diff(a) >= 0)
            o2, fl2 = oracle.ancestors_to_offspring(a)
            assert fl2 == 0 and tuple(o2) == o


def test_offspring_to_ancestors_bad_counts():
    a, fl = oracle.offspring_to_ancestors(np.array([1, 0, 1, 0]))   # sums to 2 < 4
    assert fl & oracle.FLAG_BAD_COUNTS and list(a) == [0, 2, 2, 3]
    a, fl = oracle.offspring_to_ancestors(np.array([3, 3, 0]))      # sums to 6 > 3
    assert fl & oracle.FLAG_BAD_COUNTS and list(a) == [0, 0, 0]
    a, fl = oracle.offspring_to_ancestors(np.array([-2, 3, 1]))     # negative count
    assert fl & oracle.FLAG_BAD_COUNTS and list(a) == [1, 1, 1]
    o, fl = oracle.ancestors_to_offspring(np.array([0, 5, 1]))
    assert fl & oracle.FLAG_BAD_ANCESTOR and list(o) == [1, 1, 0]


def permute_by_chains(a):
    """Code 10 computed a second way: resolve every loser's chain in the claim
    vector left by Prepermute, then assign all terminals at once."""
    n = len(a)
    d = [n] * n
    for i in range(n):
        d[a[i]] = min(d[a[i]], i)
    losers = [i for i in range(n) if d[a[i]] != i]
    term = {}
    for i in losers:
        x, seen = i, set()
        while d[x] < n:
            assert x not in seen
            seen.add(x)
            x = d[x]
        term[i] = x
    assert len(set(term.values())) == len(term)  # chains end in distinct slots
    for i, x in term.items():
        d[x] = i
    return [a[d[i]] for i in range(n)], d


def permute_random_interleaving(a, rng):
    """Code 10 with the "for each" loop run as randomly interleaved threads,
    one dependent step at a time."""
    n = len(a)
    d = [n] * n
    order = list(range(n))
    rng.shuffle(order)
    for i in order:
        d[a[i]] = min(d[a[i]], i)
    state = {}
    for i in range(n):
        if d[a[i]] != i:
            state[i] = i
    while state:
        i = rng.choice(list(state))
        x = state[i]
        if d[x] < n:
            state[i] = d[x]
        else:
            d[x] = i
            del state[i]
    return [a[d[i]] for i in range(n)]


def test_permute_brute_force():
    rng = random.Random(5)
    total = 0
    for n in range(1, 6):
        for a in itertools.product(range(n), repeat=n):
            a = list(a)
            c, fl, d = oracle.permute(np.array(a), return_d=True)
            assert fl == 0
            c = list(c)
            # a permutation of the input ancestry
            assert sorted(c) == sorted(a)
            # the predicate: o_i > 0 implies c_i = i
            for i in set(a):
                assert c[i] == i
            # a claimed slot keeps its lowest claimer (Prepermute's min rule)
            for j in set(a):
                assert d[j] == min(i for i in range(n) if a[i] == j)
            assert sorted(d) == list(range(n))  # after Permute every slot is claimed once
            c2, _ = permute_by_chains(a)
            assert c == c2
            if total % 7 == 0:
                assert c == permute_random_interleaving(a, rng)
            # Code 9 gives a (possibly different) ancestry with the same properties
            s = list(oracle.permute_serial(np.array(a)))
            assert sorted(s) == sorted(a) and all(s[i] == i for i in set(a))
            total += 1
    assert total == 1 + 4 + 27 + 256 + 3125


def test_permute_prepermute_min_rule_large():
    g = np.random.default_rng(1)
    for n in (100, 1000, 5000):
        a = g.integers(0, n, n).astype(np.int32)
        c, fl, d = oracle.permute(a, return_d=True)
        assert fl == 0
        assert sorted(c) == sorted(a)
        claimed = np.unique(a)
        assert np.all(c[claimed] == claimed)
        c2, _ = permute_by_chains(list(a))
        assert list(c) == c2


def test_permute_out_of_range_ancestors():
    c, fl = oracle.permute(np.array([1, 7, -1, 1]))
    assert fl & oracle.FLAG_BAD_ANCESTOR
    # invalid entries are replaced by their own index before permuting
    c2, fl2 = oracle.permute(np.array([1, 1, 2, 1]))
    assert fl2 == 0 and list(c) == list(c2)
