"""GPU: the autotuner tries every whole-file setting (sync mode, workgroups
per CU), every request setting (closure decode mode, one-workgroup planning
size) and re-encodes a sample per rANS lane candidate; it keeps only settings
whose output is verified, applies the fastest, and answers from its cache
the second time."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tune_and_cache(tmp_path, orc):
    import paper_2606_18900_amd as lz
    from paper_2606_18900_amd.tune import tune
    from gen.fastq import fastq
    x, _ = fastq(n_records=4000, seed=9)
    arc = lz.Archive(orc.encode(x, kind=1, level_penalty=32))
    cache = str(tmp_path / "tune.json")
    r1 = tune(arc, cache_path=cache, reps=2)
    assert not r1["cached"] and len(r1["table"]) == 6 and all(t["ok"] for t in r1["table"])
    assert r1["ms"] == min(t["ms"] for t in r1["table"])
    t = arc.tuning()
    assert (t.sync_mode, t.wg_per_cu) == (r1["sync_mode"], r1["wg_per_cu"])
    arc.set_tuning(sync_mode=1 - r1["sync_mode"])
    r2 = tune(arc, cache_path=cache)
    assert r2["cached"] and (arc.tuning().sync_mode, arc.tuning().wg_per_cu) == (r1["sync_mode"], r1["wg_per_cu"])
    out = arc.decode_all()
    torch.cuda.synchronize()
    arc.sync_status()
    assert out.cpu().numpy().tobytes() == x


def test_tune_requests(tmp_path, orc):
    import paper_2606_18900_amd as lz
    from gen.fastq import fastq
    x, starts = fastq(n_records=4000, seed=10)
    arc = lz.Archive(orc.encode(x, kind=1, level_penalty=32))
    cache = str(tmp_path / "tune.json")
    r = lz.tune_requests(arc, cache_path=cache, reps=3)
    assert not r["cached"] and len(r["table"]) == 6 and all(t["ok"] for t in r["table"])
    t = arc.tuning()
    assert (t.req_sync_mode, t.plan_blocks) == (r["req_sync_mode"], r["plan_blocks"])
    assert lz.tune_requests(arc, cache_path=cache)["cached"]
    ids = [0, 3999, 17]
    out, offs = arc.read_lookup(ids)
    torch.cuda.synchronize()
    arc.sync_status()
    o = offs.cpu().numpy()
    got = out.cpu().numpy().tobytes()
    assert [got[o[k]:o[k + 1]] for k in range(3)] == [x[starts[i]:starts[i + 1]] for i in ids]


def test_tune_encoding():
    import paper_2606_18900_amd as lz
    from gen.fastq import fastq
    x, _ = fastq(n_records=3000, seed=14)
    p = dict(kind=1, level_penalty=32)
    r = lz.tune_encoding(x, p, reps=2)
    assert len(r["table"]) == 4 and all(t["ok"] for t in r["table"])
    top = max(t["ratio"] for t in r["table"])
    assert r["ratio"] >= 0.99 * top
