"""GPU parity: whole-file decode through the C ABI must equal the oracle's
bytes (and the seeded source) exactly, in both launch modes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _decode(arc, mode, wg=2):
    print("decode_all: sync_mode %d, wg_per_cu %d, %d blocks" % (mode, wg, arc.n_blocks), flush=True)
    arc.set_tuning(sync_mode=mode, wg_per_cu=wg)
    out = arc.decode_all()
    torch.cuda.synchronize()
    arc.sync_status()
    return out.cpu().numpy().tobytes()


@pytest.fixture(scope="module")
def lz():
    import paper_2606_18900_amd as lz
    return lz


def test_config1_fastq_bit_exact(orc, lz):
    """12,000-record synthetic FASTQ, 16 KiB blocks: device bytes == oracle
    bytes == source, per-block FNV checked on the device."""
    from gen.fastq import fastq
    x, _ = fastq(n_records=12000, seed=1)
    a = orc.encode(x, kind=1, level_penalty=32)
    rc, ref = orc.decode(a)
    assert rc == 0 and ref == x
    arc = lz.Archive(a)
    for mode, wg in ((0, 2), (1, 1), (1, 2)):
        assert _decode(arc, mode, wg) == ref
    out = arc.decode_all()
    tree = int(arc.verify(out).cpu().item()) & 0xFFFFFFFFFFFFFFFF
    arc.sync_status()
    assert tree == orc.info(a).source_fnv


def _corpus():
    rng = np.random.default_rng(17)
    c = {}
    c["random4"] = rng.integers(0, 4, 5000, dtype=np.uint8).tobytes()
    c["incompressible"] = rng.integers(0, 256, 3000, dtype=np.uint8).tobytes()
    c["allsame"] = b"Q" * 4000
    for per in (1, 2, 3, 7, 61, 64, 65):
        u = rng.integers(0, 256, per, dtype=np.uint8).tobytes()
        c["period%d" % per] = (u * (4100 // per + 1))[:4100]
    motifs = [rng.integers(65, 70, 50, dtype=np.uint8).tobytes() for _ in range(6)]
    s = bytearray()
    while len(s) < 6000:
        s += motifs[int(rng.integers(0, 6))] if rng.random() < 0.6 else \
            rng.integers(65, 91, int(rng.integers(1, 40)), dtype=np.uint8).tobytes()
    c["motifs"] = bytes(s[:6000])
    return c


CORPUS = _corpus()


@pytest.mark.parametrize("name", sorted(CORPUS))
@pytest.mark.parametrize("bl,m,D", [(6, 4, 64), (8, 4, 3), (8, 6, 64)])
def test_fuzz_small_blocks(orc, lz, name, bl, m, D):
    x = CORPUS[name]
    a = orc.encode(x, block_log2=bl, min_match=m, hash_len=4, hash_bits=14, chain_depth=0,
                   max_level=D, level_penalty=2)
    rc, ref = orc.decode(a)
    assert rc == 0 and ref == x
    arc = lz.Archive(a)
    for mode in (0, 1):
        assert _decode(arc, mode) == x, (name, mode)


@pytest.mark.parametrize("lanes", [1, 64, 100, 256])
def test_fastq_lanes(orc, lz, lanes):
    from gen.fastq import fastq
    x, _ = fastq(n_records=3000, seed=5)
    a = orc.encode(x, kind=1, level_penalty=32, lit_lanes=lanes, seq_lanes=min(64, lanes))
    arc = lz.Archive(a)
    for mode in (0, 1):
        assert _decode(arc, mode) == x


def test_fasta_bit_exact(orc, lz):
    from gen.fasta import fasta
    x = fasta(4_000_000, seed=3)
    a = orc.encode(x, kind=2, level_penalty=32)
    arc = lz.Archive(a)
    for mode in (0, 1):
        assert _decode(arc, mode) == x


def test_many_in_block_matches(orc, lz):
    """Hundreds of matches per 16 KiB block whose sources lie in the block
    itself (a small vocabulary of 16..29-byte tokens), so the dependent
    in-block matches span several 64-entry chunks and many passes."""
    import numpy as np
    rng = np.random.default_rng(7)
    voc = [bytes(rng.integers(0, 256, int(rng.integers(16, 30)), dtype=np.uint8)) for _ in range(30)]
    x = b"".join(voc[i] for i in rng.integers(0, 30, 4000))
    p = dict(block_log2=14, min_match=16, hash_len=4, hash_bits=16, max_level=64, level_penalty=2)
    seqs = np.bincount(orc.parse(x, **p)["blk"])
    assert seqs.max() > 256
    arc = lz.Archive(orc.encode(x, **p))
    for mode in (0, 1):
        assert _decode(arc, mode) == x


def test_product_encoder_archive(orc, lz):
    """Archives from the library's own encoder decode to the source too."""
    from gen.fastq import fastq
    x, _ = fastq(n_records=20000, seed=8)
    a = lz.encode(x, kind=1)
    assert a == orc.encode(x, kind=1, level_penalty=32)
    arc = lz.Archive(a)
    assert _decode(arc, 1) == x


def test_empty_and_tiny(orc, lz):
    for x in (b"", b"A", b"ACGT" * 5):
        a = orc.encode(x)
        arc = lz.Archive(a)
        out = arc.decode_all()
        torch.cuda.synchronize()
        arc.sync_status()
        assert out.cpu().numpy().tobytes()[: len(x)] == x


def test_blocks_at_the_sequence_cap(orc, lz):
    """16 KiB blocks of 1024 back-to-back 16-byte matches each (the most that
    m = 16 allows), about a third of them copying from earlier matches of the
    same block: whole-file decode in both modes and range decodes equal the
    source."""
    from gen.tokens import token_stream
    x = token_stream(6)
    p = dict(block_log2=14, min_match=16, hash_len=16, hash_bits=20, max_level=64,
             level_penalty=0)
    assert list(np.bincount(orc.parse(x, **p)["blk"]))[1:] == [1024] * 5
    a = orc.encode(x, **p)
    arc = lz.Archive(a)
    for mode in (0, 1):
        assert _decode(arc, mode) == x
    B = 1 << 14
    for o, L in ((B, 3 * B), (2 * B + 5, B), (5 * B - 17, 17)):
        out = torch.empty(L + 64, dtype=torch.uint8, device="cuda")
        scratch = torch.full((arc.scratch_bytes(1),), 0xAA, dtype=torch.uint8, device="cuda")
        arc.decode_range(o, L, out=out, scratch=scratch)
        torch.cuda.synchronize()
        arc.sync_status()
        assert out[:L].cpu().numpy().tobytes() == x[o:o + L]
