"""GPU parity of the stream-separated FASTQ container (Discussion, "Where
ACEAPEX Stands on Ratio"): whole-file decode, byte ranges and read lookups
through lz_split_* must equal the oracle's plain definition (oracle/split.py)
on containers the oracle wrote, with workspace and scratch poisoned first."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

P16 = dict(block_log2=14, max_level=64, min_match=16, hash_len=16, hash_bits=18, chain_depth=16,
           window_log2=0, lit_lanes=256, seq_lanes=64, prob_bits=(12, 10, 10, 10), level_penalty=32)
P10 = dict(block_log2=10, max_level=16, min_match=16, hash_len=16, hash_bits=16, chain_depth=16,
           window_log2=0, lit_lanes=64, seq_lanes=16, prob_bits=(11, 10, 10, 10), level_penalty=4)


@pytest.fixture(scope="module")
def lz():
    import paper_2606_18900_amd as lz
    return lz


@pytest.fixture(scope="module", params=["16k", "1k"])
def split(request, lz):
    import oracle.split as sp
    from gen.fastq import fastq
    p = P16 if request.param == "16k" else P10
    x, _ = fastq(n_records=6000 if request.param == "16k" else 1500, seed=31)
    x = bytes(x)
    buf = sp.encode(x, **p)
    arc = lz.SplitArchive(buf)
    # poison the decoded-stream buffer (the front of the workspace; the stream
    # handles' own workspaces follow it)
    front = sum((int(v) + 255) // 256 * 256 for v in arc.info.stream_len)
    arc.ws[:front].fill_(0xAA)
    return x, buf, arc


def _poisoned(n, dev="cuda"):
    return torch.full((max(n, 1),), 0xAA, dtype=torch.uint8, device=dev)


def test_decode_all(split):
    import oracle.split as sp
    x, buf, arc = split
    out = arc.decode_all(_poisoned(len(x)))
    torch.cuda.synchronize()
    arc.sync_status()
    got = out.cpu().numpy().tobytes()
    assert got == sp.decode(buf)
    assert got == x


@pytest.mark.parametrize("frac", [(0.0, 1e-9), (0.0, 0.01), (0.3, 0.05), (0.5, 0.0001), (0.999, 0.001),
                                  (0.1, 0.8), (0.0, 1.0)])
def test_decode_range(split, frac):
    import oracle.split as sp
    x, buf, arc = split
    off = int(frac[0] * len(x))
    ln = max(1, min(len(x) - off, int(frac[1] * len(x))))
    sc = _poisoned(arc.scratch_bytes(1))
    out = arc.decode_range(off, ln, out=_poisoned(ln), scratch=sc)
    torch.cuda.synchronize()
    arc.sync_status()
    got = out.cpu().numpy().tobytes()
    assert got == sp.decode_range(buf, off, ln)
    assert got == x[off:off + ln]


def test_read_lookup(split):
    import oracle.split as sp
    x, buf, arc = split
    n = arc.n_reads
    rng = np.random.default_rng(5)
    ids = [0, n - 1, 7, 7, n // 2] + rng.integers(0, n, 200).tolist()
    out, offs = arc.read_lookup(ids, out=_poisoned(len(ids) * int(arc.info.max_record_len)),
                                scratch=_poisoned(arc.scratch_bytes(len(ids))))
    torch.cuda.synchronize()
    arc.sync_status()
    o = offs.cpu().numpy()
    data = out.cpu().numpy().tobytes()
    want = sp.read_lookup(buf, ids)
    assert o[0] == 0 and [int(o[k + 1] - o[k]) for k in range(len(ids))] == [len(w) for w in want]
    assert [data[int(o[k]):int(o[k + 1])] for k in range(len(ids))] == want


def test_read_lookup_out_of_range_latched(split, lz):
    x, buf, arc = split
    arc.read_lookup([0, arc.n_reads])       # the second id does not exist
    torch.cuda.synchronize()
    with pytest.raises(lz.LzError) as e:
        arc.sync_status()
    assert e.value.code == -4               # LZ_ERANGE
    arc.sync_status()                       # cleared


def test_range_outside_refused(split, lz):
    x, buf, arc = split
    with pytest.raises(lz.LzError) as e:
        arc.decode_range(len(x) - 5, 10)
    assert e.value.code == -4


def test_product_encoder_container(lz):
    from gen.fastq import fastq
    x, _ = fastq(n_records=3000, seed=32)
    x = bytes(x)
    arc = lz.SplitArchive(lz.encode_split(x, **P16))
    out = arc.decode_all()
    torch.cuda.synchronize()
    arc.sync_status()
    assert out.cpu().numpy().tobytes() == x


def test_empty_container(lz):
    import oracle.split as sp
    arc = lz.SplitArchive(sp.encode(b"", **P16))
    assert arc.n == 0 and arc.n_reads == 0
    arc.decode_all()
    torch.cuda.synchronize()
    arc.sync_status()
