"""GPU bootstrap filter (lgssm_init / lgssm_step) against the oracle.

One step: from the same device state, the GPU's ancestors equal the oracle's
(bit-exact for Metropolis and rejection, tie rule for the collective schemes),
its permutation equals Code 10 on those ancestors, and the copied, propagated
and weighted state matches the oracle's to the last bits of binary32 (the two
sides call different binary64 log/cos/exp libraries).  A captured graph of the
step replays bit-identically to eager steps.  Over a whole run, log Z-hat
agrees with the Kalman value within its Monte Carlo error.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, gpu_r_error_bound, strata_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PHI, Q, R = 0.9, 1.0, 0.5
S0 = Q / math.sqrt(1 - PHI * PHI)
SCHEMES = ["systematic", "stratified", "multinomial", "metropolis", "rejection"]


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ulp_close(a, b, ulps):
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    gap = np.abs(a.astype(np.float64) - b.astype(np.float64))
    tol = ulps * np.spacing(np.maximum(np.abs(a), np.abs(b)).astype(np.float32)).astype(np.float64)
    return np.all(gap <= tol)


def oracle_ancestors(scheme, w, B, seed, filt, t):
    if scheme == "metropolis":
        return oracle.metropolis(w, int(B), seed=seed, filt=filt, offset=t)
    if scheme == "rejection":
        return oracle.rejection(w, 1.0, seed=seed, filt=filt, offset=t)[0]
    return getattr(oracle, scheme)(w, seed=seed, filt=filt, offset=t)[0]


def check_resample(scheme, w, a_gpu, B, seed, filt, t):
    a_or = oracle_ancestors(scheme, w, B, seed, filt, t)
    if scheme in ("metropolis", "rejection"):
        assert np.array_equal(a_gpu, a_or)
        return
    n = w.size
    if scheme == "multinomial":
        _, _, r, pts = oracle.multinomial(w, seed=seed, filt=filt, offset=t, return_rp=True)
        delta = gpu_r_error_bound(w, n) + n * 2.0**-44
    else:
        _, _, r = getattr(oracle, scheme)(w, seed=seed, filt=filt, offset=t, return_r=True)
        if scheme == "stratified":
            u = oracle.stratum_offsets(n, seed=seed, filt=filt, offset=t)
        else:
            u = np.full(n, oracle.systematic_offset(seed=seed, filt=filt, offset=t))
        pts = strata_points(u)
        delta = gpu_r_error_bound(w, n)
    check_ties(a_gpu, a_or, r, pts, delta, max_ties=5 + int(20 * delta * n))


def test_init_matches_oracle():
    F, n = 3, 1000
    y = np.zeros(4)
    flt = pfr().LGSSMFilter(y, F, n, phi=PHI, q=Q, r=R, seed=7, offset=2, filter_base=5)
    flt.reset()
    x = host(flt.x)
    ref = oracle.lgssm_init(F, n, S0, seed=7, offset=2, filter_base=5)
    assert ulp_close(x, ref, 1)
    assert np.mean(x == ref) > 0.999
    assert np.all(host(flt.w) == 1.0)
    assert np.all(host(flt.log_z) == 0.0) and int(host(flt.t)[0]) == 1


@pytest.mark.parametrize("scheme", SCHEMES)
def test_steps_match_oracle(scheme):
    F, n, T = 4, 3000, 3
    y = inputs.ssm_data(T, phi=PHI, q=Q, r=R, seed=1)[1]
    flt = pfr().LGSSMFilter(y, F, n, phi=PHI, q=Q, r=R, scheme=scheme, seed=11, offset=3,
                            filter_base=2)
    flt.reset()
    for t in range(1, T + 1):
        x0, w0, lz0, B0 = host(flt.x), host(flt.w), host(flt.log_z), host(flt.B)
        flt.step()
        a, c = host(flt.ancestors), host(flt.permuted)
        for f in range(F):
            sl = slice(f * n, (f + 1) * n)
            check_resample(scheme, w0[sl].astype(np.float64), a[sl], B0[f], 11, 2 + f, t)
            assert np.array_equal(c[sl], oracle.permute(a[sl])[0])
        xo, wo, lzo, Bo = oracle.lgssm_move(c, x0, lz0, F, n, PHI, Q, R, t, y[t - 1], seed=11,
                                            offset=3, filter_base=2)
        assert ulp_close(host(flt.x), xo, 2)
        assert ulp_close(host(flt.w), wo, 4)
        np.testing.assert_allclose(host(flt.log_z), lzo, rtol=1e-12, atol=1e-12)
        check_B(host(flt.B), Bo, wo, F, n)
        assert int(host(flt.t)[0]) == t + 1
    assert int(host(flt.flags)[0]) == 0


def check_B(B_gpu, B_or, w_or, F, n):
    """B of eq. (B) per filter.  The GPU and the oracle form the weights with
    different libm calls (a few ulps apart), so their beta differ in the last
    bits and B = ceil(log eps / log(1 - beta)) may differ by one, but only
    where log eps / log(1 - beta) lies next to an integer; the resampled
    ancestors are checked with the GPU's own B."""
    diff = np.nonzero(B_gpu != B_or)[0]
    for f in diff:
        beta = float(np.mean(w_or[f * n:(f + 1) * n].astype(np.float64)))
        bstar = np.log(0.01) / np.log1p(-beta)
        assert abs(int(B_gpu[f]) - int(B_or[f])) == 1, f
        assert abs(bstar - round(bstar)) < 1e-5 * bstar, (f, bstar)


@pytest.mark.parametrize("scheme", ["systematic", "metropolis"])
def test_graph_replay_equals_eager(scheme):
    F, n, T = 8, 2048, 12
    y = inputs.ssm_data(T, phi=PHI, q=Q, r=R, seed=2)[1]
    eager = pfr().LGSSMFilter(y, F, n, phi=PHI, q=Q, r=R, scheme=scheme, seed=4)
    graph = pfr().LGSSMFilter(y, F, n, phi=PHI, q=Q, r=R, scheme=scheme, seed=4)
    lz_e = host(eager.run(graph=False))
    x_e = host(eager.x)
    for rep in range(2):  # replays after eager work in between
        lz_g = host(graph.run(graph=True))
        assert np.array_equal(lz_g, lz_e), rep
        assert np.array_equal(host(graph.x), x_e), rep
        _ = torch.ones(4, device="cuda").sum().item()


def test_step_past_last_observation_is_flagged():
    F, n, T = 2, 512, 3
    y = inputs.ssm_data(T, seed=3)[1]
    flt = pfr().LGSSMFilter(y, F, n, seed=1)
    flt.run(graph=False)
    x, lz = host(flt.x), host(flt.log_z)
    flt.step()  # t = T + 1
    assert int(host(flt.flags)[0]) == pfr().FLAG_BAD_STEP
    assert np.array_equal(host(flt.x), x) and np.array_equal(host(flt.log_z), lz)


@pytest.mark.parametrize("scheme", ["systematic", "stratified", "multinomial", "rejection"])
def test_log_likelihood_matches_kalman(scheme):
    """log Z-hat of unbiased resamplers: mean(Z-hat / Z) = 1 within 4 s.e."""
    F, n, T = 256, 4096, 50
    y = inputs.ssm_data(T, phi=PHI, q=Q, r=R, seed=0)[1]
    logZ = oracle.kalman_loglik(y, PHI, Q, R, S0)
    flt = pfr().LGSSMFilter(y, F, n, phi=PHI, q=Q, r=R, scheme=scheme, seed=9)
    lz = host(flt.run())
    ratio = np.exp(lz - logZ)
    se = ratio.std(ddof=1) / math.sqrt(F)
    assert abs(ratio.mean() - 1.0) < 4.0 * se + 1e-3, (ratio.mean(), se)
    assert int(host(flt.flags)[0]) == 0
