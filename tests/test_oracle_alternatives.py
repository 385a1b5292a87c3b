"""Pins for the oracle's Metropolis (Code 2) and rejection (Code 3) resamplers.

The law of each lane's output is known exactly for tiny n: rejection with a
first proposal j = i gives P(a_i = j) = [j = i] w_i/w_max + (1 - w_i/w_max) w_j/W;
a Metropolis lane started at i follows row i of P^B, where P is the
independent-Metropolis kernel with uniform proposals.  Replicates use
independent Philox streams (the call-offset counter word).
"""
import math
from fractions import Fraction

import numpy as np

import oracle
from lawtest import chi2_ok, frac_weights

W4 = np.array([0.5, 0.125, 0.0, 0.875])


def rejection_law(w, w_max):
    w = frac_weights(w)
    W = sum(w)
    n = len(w)
    wm = Fraction(w_max)
    P = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        acc = w[i] / wm
        for j in range(n):
            P[i][j] = (acc if i == j else 0) + (1 - acc) * w[j] / W
    return P


def metropolis_kernel(w):
    w = frac_weights(w)
    n = len(w)
    P = [[Fraction(0)] * n for _ in range(n)]
    for k in range(n):
        for j in range(n):
            if j == k:
                continue
            acc = Fraction(1) if w[k] == 0 else min(Fraction(1), w[j] / w[k])
            P[k][j] = acc / n
        P[k][k] = 1 - sum(P[k][j] for j in range(n) if j != k)
    return P


def matpow(P, B):
    n = len(P)
    R = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for _ in range(B):
        R = [[sum(R[i][m] * P[m][j] for m in range(n)) for j in range(n)] for i in range(n)]
    return R


def test_rejection_exact_marginal_law():
    K = 30000
    n = len(W4)
    counts = np.zeros((n, n))
    for rep in range(K):
        a, fl = oracle.rejection(W4, 1.0, seed=11, offset=rep)
        assert fl == 0
        counts[np.arange(n), a] += 1
    P = rejection_law(W4, 1.0)
    for i in range(n):
        ok, chi2, dof = chi2_ok(counts[i], P[i])
        assert ok, (i, chi2, dof, counts[i], [float(p) for p in P[i]])


def test_rejection_unbiased_offspring():
    # E[o_j] = n w_j / W follows from the marginal law; check it at n = 64
    w = np.random.default_rng(3).random(64) ** 3
    K = 4000
    o = np.zeros(64)
    for rep in range(K):
        a, _ = oracle.rejection(w, 1.0, seed=5, offset=rep)
        o += np.bincount(a, minlength=64)
    o /= K
    target = 64 * w / w.sum()
    # each o_j has variance <= its mean (bounded by multinomial); 6 sigma
    sd = np.sqrt(np.maximum(target, 1e-3) / K)
    assert np.all(np.abs(o - target) < 6 * sd + 1e-12)


def test_rejection_trial_counts_geometric_and_eisenberg_bound():
    # after trial 0, each trial accepts with p = W / (n w_max)
    n = 1024
    g = np.random.default_rng(8)
    w = np.exp(-0.5 * (g.standard_normal(n) - 2.0) ** 2)
    p = w.sum() / n
    maxes, tails = [], []
    for rep in range(40):
        a, fl, t = oracle.rejection(w, 1.0, seed=2, offset=rep, return_trials=True)
        assert fl == 0
        maxes.append(int(t.max()))
        tails.extend(list(t[t > 1] - 1))
    # mean number of extra trials of a lane rejected at trial 0 is 1/p
    tails = np.array(tails, dtype=np.float64)
    assert abs(tails.mean() - 1 / p) < 6 * math.sqrt((1 - p) / p**2 / tails.size)
    # expected max of n geometric(p) counts (Eisenberg 2008, section 2.2):
    # H_n / lam <= E[M] < 1 + H_n / lam with lam = -log(1 - p); lanes do at most
    # one extra (deterministic-proposal) trial, so compare the max of the tails.
    lam = -math.log(1 - p)
    H = sum(1.0 / k for k in range(1, n + 1))
    m = np.mean(maxes) - 1
    assert 0.6 * H / lam < m < 1.4 * (1 + H / lam) + 1


def test_rejection_trial_cap_and_zero_weights():
    a, fl = oracle.rejection(np.zeros(16), 1.0, max_trials=50)
    assert fl & oracle.FLAG_TRIAL_CAP
    assert np.array_equal(a, np.arange(16))
    # a zero weight is never accepted
    w = np.array([0.0, 1.0, 0.0, 0.25])
    for rep in range(200):
        a, fl = oracle.rejection(w, 1.0, offset=rep)
        assert fl == 0 and not np.any(w[a] == 0)


def test_metropolis_exact_law_of_each_lane():
    K = 30000
    B = 3
    n = len(W4)
    counts = np.zeros((n, n))
    for rep in range(K):
        a = oracle.metropolis(W4, B, seed=13, offset=rep)
        counts[np.arange(n), a] += 1
    PB = matpow(metropolis_kernel(W4), B)
    for i in range(n):
        ok, chi2, dof = chi2_ok(counts[i], PB[i])
        assert ok, (i, chi2, dof)


def test_metropolis_tv_bound_and_convergence():
    # ||P^B(i,.) - pi||_TV <= (1 - beta)^B with beta = min_i mean(w)/w_i
    w = np.array([0.5, 0.125, 0.25, 0.875])
    P = metropolis_kernel(w)
    fw = frac_weights(w)
    pi = [x / sum(fw) for x in fw]
    beta = min((sum(fw) / len(fw)) / x for x in fw)
    for B in (1, 2, 5, 10):
        PB = matpow(P, B)
        for i in range(len(w)):
            tv = sum(abs(PB[i][j] - pi[j]) for j in range(len(w))) / 2
            assert tv <= (1 - beta) ** B
    # long chains: the law of a lane approaches pi
    K = 20000
    counts = np.zeros(len(w))
    for rep in range(K):
        counts[oracle.metropolis(w, 40, seed=3, offset=rep)[0]] += 1
    ok, chi2, dof = chi2_ok(counts, pi)
    assert ok, (chi2, dof)


def test_metropolis_b_zero_is_identity():
    assert np.array_equal(oracle.metropolis(W4, 0), np.arange(4))


def test_b_star_from_bias_bound():
    # B* = log(eps) / log(1 - beta) with beta = E[w] / w_max for the paper's
    # weight sets (eps = 1/100); rounding up gives these B for y = 0..4
    from paper_1301_4019_amd.inputs import expected_weight
    B = [math.ceil(math.log(0.01) / math.log(1 - expected_weight(y))) for y in range(5)]
    assert B == [4, 6, 16, 60, 354]
