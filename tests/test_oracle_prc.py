"""Pins for the oracle's partial rejection control (section 2.2): closed
forms at the two ends of the bound, the importance weights, and the law of
the weighted offspring over many seeds."""
import numpy as np

import oracle


def test_bound_above_every_weight_is_plain_rejection_with_unit_weights():
    w = np.random.default_rng(0).exponential(size=500)
    vmax = float(w.max()) * 1.5
    a, wo, fl = oracle.partial_rejection(w, vmax, seed=3)
    assert fl == 0
    assert np.array_equal(a, oracle.rejection(w, vmax, seed=3)[0])
    assert np.all(wo == 1.0)


def test_bound_below_every_weight_keeps_every_particle():
    """v_max <= min w clips every weight to v_max, so the first proposal j = i
    is always accepted: the identity ancestry, weighted by w_i / v_max."""
    w = 2.0 + np.random.default_rng(1).exponential(size=300)
    a, wo, fl = oracle.partial_rejection(w, 2.0, seed=5)
    assert fl == 0
    assert np.array_equal(a, np.arange(300))
    assert np.array_equal(wo, w / 2.0)


def test_importance_weights_are_one_except_above_the_bound():
    w = np.random.default_rng(2).exponential(size=2000)
    vmax = float(np.quantile(w, 0.8))
    a, wo, fl = oracle.partial_rejection(w, vmax, seed=7)
    assert fl == 0
    wa = w[a]
    assert np.all(wo[wa <= vmax] == 1.0)
    assert np.array_equal(wo[wa > vmax], wa[wa > vmax] / vmax)


def test_weighted_offspring_law():
    """Code 3 with first proposal j = i gives E[o_j] = N v_j / sum(v) (each
    lane accepts i with probability v_i / v_max and otherwise draws from the
    categorical of v), so the weighted offspring sum_i w_out_i [a_i = j] has
    mean N w_j / sum(v).  Checked over 4000 seeds within 5 standard errors."""
    rng = np.random.default_rng(3)
    N = 40
    w = rng.exponential(size=N)
    w[:3] = [0.0, 4.0, 6.0]
    vmax = 1.5
    v = np.minimum(w, vmax)
    expect = N * w / v.sum()
    K = 4000
    acc = np.zeros((K, N))
    for k in range(K):
        a, wo, fl = oracle.partial_rejection(w, vmax, seed=100 + k)
        assert fl == 0
        np.add.at(acc[k], a, wo)
    mean = acc.mean(axis=0)
    se = acc.std(axis=0, ddof=1) / np.sqrt(K)
    assert mean[0] == 0.0
    assert np.all(np.abs(mean - expect) <= 5 * se + 1e-12), np.max(np.abs(mean - expect) / (se + 1e-12))


def test_trial_cap_on_a_zero_weight():
    a, wo, fl = oracle.partial_rejection(np.array([0.0, 1.0, 1.0]), 1.0, seed=1, max_trials=1)
    assert fl == oracle.FLAG_TRIAL_CAP
    assert a[0] == 0 and wo[0] == 0.0
