"""Host logic of the served decode loop, with a stand-in lane that serves from
the source bytes: admission in arrival order, windows of long ranges, batch
limits (request count and output bytes), budget check, every request's bytes
assembled exactly, latencies non-negative."""
import numpy as np
import pytest

from gen.requests import poisson_trace
from paper_2606_18900_amd.serve import Server


class _Info:
    block_log2 = 10


class FakeArc:
    def __init__(self, x):
        self.x = x
        self.n = len(x)
        self.info = _Info()
        self.n_blocks = (len(x) + 1023) // 1024

    def scratch_bytes(self, n, slots):
        return 64 * n + slots * 1024


class _Ev:
    def query(self):
        return True


class FakeLane:
    log = []

    def __init__(self, arc, n_max, out_cap, n_slots=None, use_graph=True, stream=None, scratch=None):
        self.arc, self.n_max, self.cap = arc, n_max, out_cap
        self.res = []
        self.starts = None

    def submit(self, kind, a, b):
        assert len(kind) <= self.n_max
        out = []
        for k, aa, bb in zip(kind, a, b):
            if k == 0:
                s = FakeLane.starts
                out.append(self.arc.x[s[aa]:s[aa + 1]])
            else:
                out.append(self.arc.x[aa:aa + bb])
        assert sum(len(o) for o in out) <= self.cap
        FakeLane.log.append((len(kind), sum(len(o) for o in out)))
        self.res = out

    def event(self, timing=False):
        return _Ev()

    def synchronize(self):
        pass

    def results(self):
        return self.res


def _source(n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, n, dtype=np.uint8).tobytes()


def test_serve_host_exact():
    xq = _source(200_000, 1)
    starts = np.unique(np.concatenate([[0], np.sort(np.random.default_rng(2).choice(np.arange(1, 200_000), 800, replace=False)), [200_000]])).astype(np.int64)
    xg = _source(300_000, 3)
    FakeLane.starts = starts
    FakeLane.log = []
    tr = poisson_trace(20000.0, 0.02, starts, len(xq), len(xg), seed=7, big_range=100_000)
    srv = Server([FakeArc(xq), FakeArc(xg)], [starts, None], budget=64 << 20, lanes=2,
                 n_max=8, window=30_000, keep_results=True, batcher=FakeLane)
    res = srv.run(tr)
    assert res["completed"] == res["offered"] == len(tr["t"])
    for rid, got in res["results"].items():
        k, kind, a, b = (int(tr[f][rid]) for f in ("archive", "kind", "a", "b"))
        want = xq[starts[a]:starts[a + 1]] if kind == 0 else (xq, xg)[k][a:a + b]
        assert got == want
    assert max(n for n, _ in FakeLane.log) <= 8
    assert max(by for _, by in FakeLane.log) <= 30_000
    assert res["p50_ms"] >= 0


def test_serve_host_budget():
    x = _source(50_000, 4)
    with pytest.raises(ValueError):
        Server([FakeArc(x)], [None], budget=1000, lanes=1, n_max=4, window=4096, batcher=FakeLane)


def test_serve_host_refuses_read_larger_than_window():
    """A read whose record cannot fit one window is refused with LZ_EBUDGET
    (it could never be served within the budget) instead of being queued
    forever; every other request is still served exactly."""
    from paper_2606_18900_amd._lib import LZ_EBUDGET
    x = _source(100_000, 5)
    starts = np.array([0, 1000, 9000, 9500, 100_000], dtype=np.int64)   # record 3 is 90,500 bytes
    FakeLane.starts = starts
    tr = {"t": np.array([0.0, 0.0, 0.0, 0.0]), "archive": np.zeros(4, dtype=np.int64),
          "kind": np.zeros(4, dtype=np.int64), "a": np.array([0, 1, 2, 3]), "b": np.zeros(4, dtype=np.int64)}
    srv = Server([FakeArc(x)], [starts], budget=64 << 20, lanes=2, n_max=4, window=10_000,
                 keep_results=True, batcher=FakeLane)
    res = srv.run(tr)
    assert res["completed"] == 3 and res["refused"] == {"LZ_EBUDGET": 1}
    assert res["refused_ids"] == {3: LZ_EBUDGET}
    for rid in (0, 1, 2):
        assert res["results"][rid] == x[starts[rid]:starts[rid + 1]]


class _NeverEv:
    def query(self):
        return False


class StuckLane(FakeLane):
    def event(self, timing=False):
        return _NeverEv()


def test_serve_host_stall_raises():
    """A loop that cannot make progress (a batch that never completes) raises
    after stall_s instead of spinning forever."""
    x = _source(50_000, 6)
    tr = {"t": np.array([0.0]), "archive": np.zeros(1, dtype=np.int64), "kind": np.ones(1, dtype=np.int64),
          "a": np.array([0]), "b": np.array([1000])}
    srv = Server([FakeArc(x)], [None], budget=64 << 20, lanes=1, n_max=4, window=4096,
                 batcher=StuckLane, stall_s=0.5)
    with pytest.raises(RuntimeError):
        srv.run(tr)
