"""GPU: the served decode loop (continuous batching over two resident archives,
capped output windows, budget) returns every request's bytes exactly: reads
and ranges checked against the seeded sources, for batched and one-request-
per-launch serving."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    import paper_2606_18900_amd as lz
    from gen.fasta import fasta
    from gen.fastq import fastq
    xq, starts = fastq(n_records=6000, seed=5)
    xg = fasta(3 << 20, seed=3)
    aq = lz.encode(xq, kind=1, level_penalty=32, hash_bits=22, block_log2=14)
    ag = lz.encode(xg, kind=2, level_penalty=32, hash_bits=22, block_log2=14)
    return lz, xq, np.asarray(starts, dtype=np.int64), xg, lz.Archive(aq), lz.Archive(ag)


def _check(res, trace, xq, starts, xg):
    src = (xq, xg)
    assert res["completed"] == res["offered"]
    for rid, got in res["results"].items():
        k, kind, a, b = (int(trace[f][rid]) for f in ("archive", "kind", "a", "b"))
        if kind == 0:
            want = xq[int(starts[a]):int(starts[a + 1])]
        else:
            want = src[k][a:a + b]
        assert got == want, (rid, k, kind, a, b)


@pytest.mark.parametrize("lanes,n_max,graph", [(3, 64, True), (1, 1, False)])
def test_serve_exact(setup, lanes, n_max, graph):
    lz, xq, starts, xg, arq, arg = setup
    from gen.requests import poisson_trace
    from paper_2606_18900_amd.serve import Server
    tr = poisson_trace(3000.0, 0.1, starts, len(xq), len(xg), seed=5, big_range=1 << 20)
    # windows smaller than the large ranges, so those are served in pieces
    srv = Server([arq, arg], [starts, None], budget=2 << 30, lanes=lanes, n_max=n_max,
                 window=256 << 10, use_graph=graph, keep_results=True)
    res = srv.run(tr, time_limit_s=60)
    _check(res, tr, xq, starts, xg)
    assert res["p50_ms"] is not None and res["p99_ms"] >= res["p50_ms"]


def test_serve_budget_too_small(setup):
    lz, xq, starts, xg, arq, arg = setup
    from paper_2606_18900_amd.serve import Server
    with pytest.raises(ValueError):
        Server([arq, arg], [starts, None], budget=1 << 20, lanes=2, n_max=16, window=256 << 10)


def test_serve_overlap_and_isolation(setup):
    """Lanes run on their own streams and handles: batches admitted while
    another batch is on the device start before it ends (device events), and
    every request returns the same bytes in the mix as when served alone
    (both equal to the plain definition)."""
    lz, xq, starts, xg, arq, arg = setup
    from paper_2606_18900_amd.serve import Server
    rng = np.random.default_rng(21)
    n = 40
    t = np.concatenate([[0.0, 0.0], np.sort(rng.uniform(0.0005, 0.004, n - 2))])
    arch = np.concatenate([[1, 1], rng.integers(0, 2, n - 2)])
    kind = np.where(arch == 0, 0, 1)
    kind[:2] = 1
    a = np.where(kind == 0, rng.integers(0, len(starts) - 1, n), rng.integers(0, len(xg) - (1 << 18), n))
    b = np.where(kind == 0, 0, rng.integers(1 << 12, 1 << 18, n))
    a[:2], b[:2] = [0, 1 << 20], [len(xg) - (1 << 20), len(xg) - (1 << 20)]   # two long ranges first
    tr = {"t": t, "archive": arch, "kind": kind, "a": a.astype(np.int64), "b": b.astype(np.int64)}
    srv = Server([arq, arg], [starts, None], budget=2 << 30, lanes=3, n_max=8, window=4 << 20,
                 keep_results=True)
    res = srv.run(tr, time_limit_s=60)
    _check(res, tr, xq, starts, xg)
    ov = res["device_overlap"]
    assert ov["started_while_another_ran"] >= 1 and ov["max_concurrent"] >= 2, ov
    # a batch holding requests admitted after the first batch was launched
    # starts on the device before that first batch ends
    iv = srv.intervals()
    first = iv[0]
    assert any(s < first[3] and min(r for r in rids) >= 2 for _, _, s, _, rids in iv[1:]), iv[:6]
    # alone: each of the first eight requests served by itself
    solo = Server([arq, arg], [starts, None], budget=2 << 30, lanes=1, n_max=1, window=4 << 20,
                  keep_results=True)
    for rid in range(8):
        one = {f: tr[f][rid:rid + 1] for f in ("archive", "kind", "a", "b")}
        one["t"] = np.zeros(1)
        r1 = solo.run(one, time_limit_s=30)
        assert r1["results"][0] == res["results"][rid]
