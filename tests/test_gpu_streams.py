"""Calls enqueued on several HIP streams at once: the binding keeps one cached
workspace per stream, so concurrent calls of the same operation and size do
not share claim vectors, records or bound tables.  Every result must equal
the oracle's, as for calls on one stream."""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from test_gpu_parity import check_collective

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def test_concurrent_streams_same_size():
    n = 1 << 18
    ys = (0.5, 2.0, 3.5)
    ws = [inputs.weights(n, y, seed=40 + k) for k, y in enumerate(ys)]
    wd = [torch.from_numpy(w).cuda() for w in ws]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in ys]
    res = []
    # three rounds, so that the calls of one round overlap those of the others
    for rnd in range(3):
        for k, st in enumerate(streams):
            with torch.cuda.stream(st):
                a_rej = pfr().resample_rejection(wd[k], 1.0, seed=rnd)
                c_rej = pfr().permute_ancestors(a_rej)
                a_met = pfr().resample_metropolis(wd[k], 20, seed=rnd)
                a_sys, c_sys = pfr().resample_permuted("systematic", wd[k], seed=rnd)
                a_mul = pfr().resample_multinomial(wd[k], seed=rnd)
                res.append((rnd, k, a_rej, c_rej, a_met, a_sys, c_sys, a_mul))
    torch.cuda.synchronize()
    for rnd, k, a_rej, c_rej, a_met, a_sys, c_sys, a_mul in res:
        w = ws[k]
        ref_rej = oracle.rejection(w, 1.0, seed=rnd)[0]
        assert np.array_equal(a_rej.cpu().numpy(), ref_rej), (rnd, k)
        assert np.array_equal(c_rej.cpu().numpy(), oracle.permute(ref_rej)[0]), (rnd, k)
        assert np.array_equal(a_met.cpu().numpy(), oracle.metropolis(w, 20, seed=rnd)), (rnd, k)
        # collective schemes: the oracle's answer up to the stated boundary ties
        got_sys = a_sys.cpu().numpy()
        check_collective("systematic", w, got_sys, seed=rnd)
        assert np.array_equal(c_sys.cpu().numpy(), oracle.permute(got_sys)[0]), (rnd, k)
        check_collective("multinomial", w, a_mul.cpu().numpy(), seed=rnd)
