"""Host-side logic of the Python binding (no GPU): the workspace cache keeps
at most its byte budget, dropping the least recently used workspace first."""
from paper_1301_4019_amd import _WorkspaceCache


class FakeWs:
    def __init__(self, nbytes):
        self.nbytes = nbytes

    def numel(self):
        return self.nbytes


def test_workspace_cache_evicts_least_recently_used():
    c = _WorkspaceCache(100)
    a, b, d = FakeWs(40), FakeWs(40), FakeWs(40)
    c.put("a", a)
    c.put("b", b)
    assert c.get("a") is a  # a is now the most recent
    c.put("d", d)           # over budget: b goes
    assert c.get("b") is None and c.get("a") is a and c.get("d") is d
    assert c.bytes == 80


def test_workspace_cache_keeps_one_oversized_entry():
    c = _WorkspaceCache(10)
    big = FakeWs(1000)
    c.put("big", big)
    assert c.get("big") is big and c.bytes == 1000
    c.put("small", FakeWs(5))
    assert c.get("big") is None and c.bytes == 5
    c.clear()
    assert c.bytes == 0 and c.get("small") is None
