"""GPU: the launch autotuner tries every (sync mode, workgroups per CU),
keeps only settings whose output reproduces the source hash, applies the
fastest, and answers from its cache the second time."""
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
    assert not r1["cached"] and len(r1["table"]) == 8 and all(t["ok"] for t in r1["table"])
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
