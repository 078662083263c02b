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
