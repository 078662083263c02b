"""GPU test of the allocation-free read lookup: its output equals that of
lz_read_lookup (caller-provided scratch) and the plain definition (the 4-line
records), on two calls in a row, the second with fewer ids."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_read_lookup_matches_read_lookup(orc):
    import paper_2606_18900_amd as lz
    from paper_2606_18900_amd import _lib
    from gen.fastq import fastq
    x, starts = fastq(n_records=12000, seed=1)
    a = orc.encode(x, kind=1, level_penalty=32)
    arc = lz.Archive(a)
    rng = np.random.default_rng(11)
    mr = int(arc.info.max_record_len)
    for n in (3000, 17):                      # second call smaller than the first
        ids_h = rng.integers(0, arc.n_reads, n)
        ids_h[: min(n, 5)] = ids_h[0]         # duplicates keep request order
        ids = torch.as_tensor(ids_h, dtype=torch.int64, device="cuda")
        out_a = torch.full((n * mr,), 0x55, dtype=torch.uint8, device="cuda")
        off_a = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        arc.read_lookup_noalloc(ids, out_a, off_a)
        torch.cuda.synchronize()
        arc.sync_status()
        out_b, off_b = arc.read_lookup(ids)
        torch.cuda.synchronize()
        arc.sync_status()
        oa, ob = off_a.cpu().numpy(), off_b.cpu().numpy()
        assert np.array_equal(oa, ob)
        tot = int(oa[-1])
        ga = out_a[:tot].cpu().numpy().tobytes()
        assert ga == out_b[:tot].cpu().numpy().tobytes()
        want = b"".join(x[starts[r]:starts[r + 1]] for r in ids_h)
        assert ga == want


def test_noalloc_rejects_too_many_ids(orc):
    import paper_2606_18900_amd as lz
    from paper_2606_18900_amd import _lib
    from gen.fastq import fastq
    x, starts = fastq(n_records=2000, seed=1)
    arc = lz.Archive(orc.encode(x, kind=1, level_penalty=32))
    n = _lib.NOALLOC_MAX_IDS + 1
    ids = torch.zeros(n, dtype=torch.int64, device="cuda")
    out = torch.empty(n * int(arc.info.max_record_len), dtype=torch.uint8, device="cuda")
    offs = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(_lib.LzError) as e:
        arc.read_lookup_noalloc(ids, out, offs)
    assert e.value.code == _lib.LZ_ECAPACITY
