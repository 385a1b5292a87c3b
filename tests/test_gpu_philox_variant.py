"""The Philox round-count study build (libpfresample_philox7.so) against the
oracle run with the same round count: every resampler draws through the
one Philox function, so parity with 7 rounds shows that the round count is
the only difference between the builds.  The product build reports 10."""
import os

import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, gpu_r_error_bound, strata_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def variant():
    from paper_1301_4019_amd import build
    path = build.variant_path(7)
    if not os.path.exists(path):
        pytest.fail(f"{path} is not built (python -m paper_1301_4019_amd.build)")
    return path


def test_product_build_uses_ten_rounds():
    assert pfr()._lib.load().pfr_philox_rounds() == 10


@pytest.mark.parametrize("n", [1000, 1 << 18])
def test_seven_round_build_matches_the_oracle(n):
    w = inputs.weights(n, 2.0, seed=n)
    wd = torch.from_numpy(w).cuda()
    with pfr()._lib.use_library(variant()) as lib:
        assert lib.pfr_philox_rounds() == 7
        am = host(pfr().resample_metropolis(wd, 16, seed=2))
        ar = host(pfr().resample_rejection(wd, 1.0, seed=2))
        ast = host(pfr().resample_stratified(wd, seed=2))
        ai = host(pfr().resample_multinomial_iid(wd, seed=2))
    a10 = host(pfr().resample_metropolis(wd, 16, seed=2))
    assert not np.array_equal(am, a10)
    with oracle.philox_rounds(7):
        assert np.array_equal(am, oracle.metropolis(w, 16, seed=2))
        assert np.array_equal(ar, oracle.rejection(w, 1.0, seed=2)[0])
        _, _, r = oracle.stratified(w, seed=2, return_r=True)
        a_or = oracle.stratified(w, seed=2)[0]
        pts = strata_points(oracle.stratum_offsets(n, seed=2))
        delta = gpu_r_error_bound(w.astype(np.float64), n)
        check_ties(ast, a_or, r, pts, delta, max_ties=5 + int(20 * delta * n))
        ai_or, _, ri, pi = oracle.multinomial_iid(w, seed=2, return_rp=True)
        check_ties(ai, ai_or, ri, pi, delta, max_ties=5 + int(20 * delta * n))
