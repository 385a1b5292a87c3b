"""The precondition checks (pfr_set_checks): violations are flagged, a wrong
sorted_hint no longer changes the permutation, and valid inputs give the same
bits with the checks on as with them off."""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def new_flags():
    return torch.zeros(1, dtype=torch.int32, device="cuda")


@pytest.fixture
def checks():
    """The checks on for one test (the setting is process-wide), with the
    library's check word cleared before and after."""
    m = pfr()
    m.set_checks(True)
    m.take_check_flags()
    try:
        yield m
    finally:
        m.take_check_flags()
        m.set_checks(False)


def test_switch():
    m = pfr()
    assert not m.get_checks()
    m.set_checks(True)
    try:
        assert m.get_checks()
    finally:
        m.set_checks(False)
    assert not m.get_checks()


@pytest.mark.parametrize("n", [5000, (1 << 17) + 3])
def test_valid_inputs_unchanged(n):
    m = pfr()
    w = inputs.weights(n, 3.0, seed=n)
    wd = dev(w)
    asys = host(m.resample_systematic(wd, seed=4))
    off = dict(a=m.resample_metropolis(wd, 60, seed=3), r=m.resample_rejection(wd, 1.0, seed=3),
               c=m.permute_ancestors(dev(asys), sorted_hint=True),
               k=m.permute_ancestors_noalloc(dev(asys), sorted_hint=True),
               o=m.ancestors_to_offspring(dev(asys), sorted_hint=True))
    off = {k: host(v) for k, v in off.items()}
    m.set_checks(True)
    try:
        m.take_check_flags()
        fl = new_flags()
        on = dict(a=m.resample_metropolis(wd, 60, seed=3),
                  r=m.resample_rejection(wd, 1.0, seed=3, flags=fl),
                  c=m.permute_ancestors(dev(asys), sorted_hint=True, flags=fl),
                  k=m.permute_ancestors_noalloc(dev(asys), sorted_hint=True, flags=fl),
                  o=m.ancestors_to_offspring(dev(asys), sorted_hint=True, flags=fl))
        on = {k: host(v) for k, v in on.items()}
        assert m.take_check_flags() == 0
    finally:
        m.set_checks(False)
    assert int(host(fl)[0]) == 0
    for k in off:
        assert np.array_equal(on[k], off[k]), k
    assert np.array_equal(off["c"], oracle.permute(asys)[0])


@pytest.mark.parametrize("n", [5000, (1 << 17) + 3])
def test_wmax_below_a_weight(checks, n):
    m = checks
    w = inputs.weights(n, 0.0, seed=n)  # maximum close to 1
    wd = dev(w)
    fl = new_flags()
    a = host(m.resample_rejection(wd, 0.5, seed=8, flags=fl))
    assert int(host(fl)[0]) & m.FLAG_WMAX_BELOW
    assert m.take_check_flags() & m.FLAG_WMAX_BELOW
    m.set_checks(False)
    ref = host(m.resample_rejection(wd, 0.5, seed=8))
    assert np.array_equal(a, ref)  # the check flags, it does not change the output
    # a bound equal to the largest weight is valid
    m.set_checks(True)
    fl = new_flags()
    m.resample_rejection(wd, float(w.max()), seed=8, flags=fl)
    assert int(host(fl)[0]) & m.FLAG_WMAX_BELOW == 0
    assert m.take_check_flags() == 0


def test_wmax_per_segment(checks):
    m = checks
    lens = [3000, 4000, 2500]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([inputs.weights(k, 0.0, seed=k) for k in lens])
    bounds = np.array([w[off[f]:off[f + 1]].max() for f in range(3)], dtype=np.float64)
    fl = new_flags()
    m.resample_rejection(dev(w), 1.0, seed=2, w_max_per_filter=dev(bounds), offsets=dev(off),
                         max_len=max(lens), flags=fl)
    assert int(host(fl)[0]) == 0 and m.take_check_flags() == 0
    low = bounds.copy()
    low[2] *= 0.75  # only the last segment's bound is too small
    fl = new_flags()
    m.resample_rejection(dev(w), 1.0, seed=2, w_max_per_filter=dev(low), offsets=dev(off),
                         max_len=max(lens), flags=fl)
    assert int(host(fl)[0]) & m.FLAG_WMAX_BELOW
    assert m.take_check_flags() & m.FLAG_WMAX_BELOW


@pytest.mark.parametrize("n", [5000, (1 << 17) + 3])
def test_bad_weights_metropolis_and_rejection(checks, n):
    m = checks
    w = inputs.weights(n, 2.0, seed=n)
    w[5] = np.nan
    w[n // 2] = -1.0
    m.resample_metropolis(dev(w), 60, seed=1)
    assert m.take_check_flags() & m.FLAG_BAD_WEIGHTS
    w = inputs.weights(n, 2.0, seed=n)
    w[n - 1] = np.inf
    fl = new_flags()
    m.resample_rejection(dev(w), 1.0, seed=1, max_trials=64, flags=fl)
    assert int(host(fl)[0]) & m.FLAG_BAD_WEIGHTS
    assert m.take_check_flags() & m.FLAG_BAD_WEIGHTS


@pytest.mark.parametrize("n", [5000, (1 << 18) + 3])
def test_sorted_hint_on_unsorted_ancestry(checks, n):
    m = checks
    g = np.random.default_rng(n)
    p = g.random(n) ** 4
    a = g.choice(n, size=n, p=p / p.sum()).astype(np.int32)
    ref, _ = oracle.permute(a)
    fl = new_flags()
    c = host(m.permute_ancestors(dev(a), sorted_hint=True, flags=fl))
    assert np.array_equal(c, ref)
    assert int(host(fl)[0]) & m.FLAG_NOT_SORTED
    fl = new_flags()
    c = host(m.permute_ancestors_noalloc(dev(a), sorted_hint=True, flags=fl))
    assert np.array_equal(c, ref)
    assert int(host(fl)[0]) & m.FLAG_NOT_SORTED
    fl = new_flags()
    o = host(m.ancestors_to_offspring(dev(a), sorted_hint=True, flags=fl))
    assert np.array_equal(o, np.bincount(a, minlength=n))
    assert int(host(fl)[0]) & m.FLAG_NOT_SORTED
    assert m.take_check_flags() == m.FLAG_NOT_SORTED
    assert m.take_check_flags() == 0  # taking clears the word


def test_sorted_hint_segments(checks):
    """A step down at a segment start is allowed; one inside a segment is not."""
    m = checks
    lens = [7000, 1, 9000, 3000]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    g = np.random.default_rng(5)
    segs = [np.sort(g.integers(0, k, k)).astype(np.int32) for k in lens]
    a = np.concatenate(segs)
    refs = [oracle.permute(s)[0] for s in segs]
    fl = new_flags()
    c = host(m.permute_ancestors(dev(a), sorted_hint=True, offsets=dev(off), max_len=max(lens),
                                 flags=fl))
    assert int(host(fl)[0]) == 0 and m.take_check_flags() == 0
    assert np.array_equal(c, np.concatenate(refs))
    segs[2] = segs[2][::-1].copy()  # one unsorted segment
    a = np.concatenate(segs)
    refs[2] = oracle.permute(segs[2])[0]
    fl = new_flags()
    c = host(m.permute_ancestors(dev(a), sorted_hint=True, offsets=dev(off), max_len=max(lens),
                                 flags=fl))
    assert int(host(fl)[0]) & m.FLAG_NOT_SORTED
    assert m.take_check_flags() & m.FLAG_NOT_SORTED
    assert np.array_equal(c, np.concatenate(refs))
