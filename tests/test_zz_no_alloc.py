"""The no-allocation permutation against permute_ancestors (Code 10).

permute_ancestors_noalloc keeps its claim vector and marks in the library's
static device scratch instead of a caller workspace.  Its output must equal
permute_ancestors' bit for bit (integer work), on calls in a row whose sizes
shrink (the scratch keeps the previous call's contents), on sorted and
unsorted ancestries, on a batch, and at the largest size it accepts; the
oracle's Code 10 pins the small cases.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import _lib

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def ancestry(n, seed, sorted_, parents=None):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, parents or n, size=n, dtype=np.int64).astype(np.int32)
    return np.sort(a) if sorted_ else a


def both(a_np, sorted_, offsets=None, max_len=None):
    a = torch.from_numpy(a_np).cuda()
    off = None if offsets is None else torch.from_numpy(offsets).cuda()
    fl0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    fl1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = pfr().permute_ancestors(a, sorted_hint=sorted_, offsets=off, max_len=max_len,
                                  flags=fl0)
    out = torch.full_like(a, -7)
    got = pfr().permute_ancestors_noalloc(a, sorted_hint=sorted_, offsets=off, max_len=max_len,
                                          out=out, flags=fl1)
    assert got.data_ptr() == out.data_ptr()
    return host(ref), host(got), int(host(fl0)[0]), int(host(fl1)[0])


@pytest.mark.parametrize("sorted_", [False, True])
def test_two_calls_in_a_row_second_smaller(sorted_):
    for n, seed in ((3_000_001, 1), (200_003, 2)):
        ref, got, f0, f1 = both(ancestry(n, seed, sorted_), sorted_)
        assert f0 == f1 == 0
        assert np.array_equal(got, ref), n


def test_largest_accepted_size_then_small_with_oracle():
    n = _lib.NOALLOC_MAX_N
    ref, got, f0, f1 = both(ancestry(n, 3, False, parents=n // 16), False)
    assert f0 == f1 == 0 and np.array_equal(got, ref)
    a = ancestry(50_000, 4, False)
    ref, got, f0, f1 = both(a, False)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.permute(a)[0])


def test_batch_and_bad_ancestor_flag():
    lens = np.array([7, 20_000, 1, 70_000, 300], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    parts = [ancestry(int(m), 10 + k, False) for k, m in enumerate(lens)]
    parts[2][0] = 5  # out of range for a segment of one: treated as its own index
    a = np.concatenate(parts)
    ref, got, f0, f1 = both(a, False, offsets=off, max_len=int(lens.max()))
    assert f0 == f1 == _lib.FLAG_BAD_ANCESTOR
    assert np.array_equal(got, ref)
    for k in range(lens.size):
        sl = slice(off[k], off[k + 1])
        assert np.array_equal(got[sl], oracle.permute(a[sl])[0]), k


def test_rejects_beyond_the_scratch_and_enqueues_nothing():
    n = _lib.NOALLOC_MAX_N + 1
    a = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.full_like(a, -3)
    seg = _lib.Segments(n, 1, None, n)
    rc = _lib.load().permute_ancestors_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.byref(seg), 0,
                                               ctypes.c_void_p(out.data_ptr()), None,
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.PFR_ETOOBIG
    assert int((out != -3).sum().item()) == 0
