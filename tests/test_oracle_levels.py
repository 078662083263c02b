"""Pins for the oracle's level-parallel decoder (the CPU baseline the benchmark
times): at one thread and at several it must return exactly the seeded source
and the sequential decoder's bytes, on archives with many dependency levels,
on the small-block corpus and on the 12,000-record FASTQ; and it must reject a
block whose sources lie outside its dependency list, as the sequential
decoder does.  Also the token stream that puts blocks at the sequence cap."""
import numpy as np
import pytest

from tests.ref.tamper import swap_dependency


def _levels(orc, a, n, threads):
    out = np.full(max(n, 1), 0xAA, dtype=np.uint8)
    rc = orc.decode_levels(a, out, threads)
    return rc, out[:n].tobytes()


def _deep(orc):
    rng = np.random.default_rng(3)
    motifs = [rng.integers(65, 70, 50, dtype=np.uint8).tobytes() for _ in range(6)]
    s = bytearray()
    while len(s) < 40000:
        s += motifs[int(rng.integers(0, 6))] if rng.random() < 0.6 else \
            rng.integers(65, 91, int(rng.integers(1, 40)), dtype=np.uint8).tobytes()
    x = bytes(s[:40000])
    a = orc.encode(x, block_log2=6, min_match=4, hash_len=4, hash_bits=14, max_level=64,
                   level_penalty=0)
    return x, a


@pytest.mark.parametrize("threads", [1, 2, 8])
def test_levels_deep_archive(orc, threads):
    x, a = _deep(orc)
    assert orc.info(a).n_levels >= 5
    rc, ref = orc.decode(a)
    assert rc == 0 and ref == x
    rc, got = _levels(orc, a, len(x), threads)
    assert rc == 0 and got == x


@pytest.mark.parametrize("threads", [1, 4])
def test_levels_fastq_config1(orc, threads):
    from gen.fastq import fastq
    x, _ = fastq(n_records=12000, seed=1)
    a = orc.encode(x, kind=1, level_penalty=32)
    assert orc.info(a).n_levels >= 5
    rc, got = _levels(orc, a, len(x), threads)
    assert rc == 0 and got == x


def test_levels_corpus(orc):
    rng = np.random.default_rng(17)
    cases = [rng.integers(0, 4, 5000, dtype=np.uint8).tobytes(), b"Q" * 4000,
             (rng.integers(0, 256, 7, dtype=np.uint8).tobytes() * 700)[:4100]]
    for x in cases:
        for bl, m, D in ((6, 4, 64), (8, 4, 3)):
            a = orc.encode(x, block_log2=bl, min_match=m, hash_len=4, hash_bits=14,
                           chain_depth=0, max_level=D, level_penalty=2)
            for threads in (1, 3):
                rc, got = _levels(orc, a, len(x), threads)
                assert rc == 0 and got == x


def test_levels_rejects_source_outside_dependencies(orc):
    from gen.fastq import fastq
    x, _ = fastq(n_records=3000, seed=1)
    t, b, d, d2 = swap_dependency(orc.encode(x, kind=1, level_penalty=32))
    assert orc.validate(t) == 0                 # lists, levels and header are consistent
    assert orc.decode(t)[0] == orc.ECORRUPT
    for threads in (1, 4):
        assert _levels(orc, t, len(x), threads)[0] == orc.ECORRUPT
    rc, _, _ = orc.decode_range(t, b << 14, 100)
    assert rc == orc.ECORRUPT


def test_token_stream_fills_the_sequence_cap(orc):
    """Every block after the first: 1024 sequences of LL = 0, ML = 16 (the most
    that B = 16 KiB and m = 16 allow), many with sources in their own block."""
    from gen.tokens import token_stream
    x = token_stream(4)
    p = dict(block_log2=14, min_match=16, hash_len=16, hash_bits=20, max_level=64,
             level_penalty=0)
    r = orc.parse(x, **p)
    per = np.bincount(r["blk"])
    assert list(per) == [1, 1024, 1024, 1024]
    assert set(r["ml"][r["blk"] > 0].tolist()) == {16}
    assert set(r["ll"][r["blk"] > 0].tolist()) == {0}
    inblock = (r["of"] >= (r["blk"].astype(np.uint64) << np.uint64(14))).sum()
    assert inblock > 500
    rc, out = orc.decode(orc.encode(x, **p))
    assert rc == 0 and out == x
