"""The library's host encoder (lz_encode) and the oracle's encoder are
independent implementations of the same policy: their archives must be
byte-identical, single- and multi-threaded, for every parameter shape."""
import numpy as np
import pytest

lz = pytest.importorskip("paper_2606_18900_amd")


@pytest.fixture(scope="module")
def have_lib():
    try:
        lz.lib()
    except RuntimeError as e:
        pytest.skip(str(e))


PARAMS = [
    dict(block_log2=6, min_match=4, hash_len=4, hash_bits=12, chain_depth=0, window_log2=0,
         max_level=64, level_penalty=0),
    dict(block_log2=8, min_match=5, hash_len=4, hash_bits=12, chain_depth=3, window_log2=7,
         max_level=3, level_penalty=2),
    dict(block_log2=6, min_match=4, hash_len=4, hash_bits=10, chain_depth=0, window_log2=0,
         max_level=64, level_penalty=3),
    dict(block_log2=10, min_match=8, hash_len=6, hash_bits=16, chain_depth=8, window_log2=0,
         max_level=8, level_penalty=8, lit_lanes=100, seq_lanes=7, prob_bits=(9, 8, 11, 12)),
]


def test_identical_on_parse_inputs(orc, have_lib):
    from tests.test_oracle_parse import INPUTS
    for name, x in INPUTS.items():
        for kw in PARAMS:
            ref = orc.encode(x, **kw)
            for t in (1, 3):
                assert lz.encode(x, threads=t, **kw) == ref, (name, kw, t)


def test_identical_fastq_and_fasta(orc, have_lib):
    from gen.fasta import fasta
    from gen.fastq import fastq
    x, _ = fastq(n_records=12000, seed=1)
    assert lz.encode(x, kind=1) == orc.encode(x, kind=1, level_penalty=32)
    assert lz.encode(x, kind=1, hash_bits=24, chain_depth=16, threads=4) == \
        orc.encode(x, kind=1, hash_bits=24, chain_depth=16, level_penalty=32)
    g = fasta(2_000_000, seed=3)
    assert lz.encode(g, kind=2, window_log2=12, chain_depth=8) == \
        orc.encode(g, kind=2, window_log2=12, chain_depth=8, level_penalty=32)


def test_encoder_rejects_bad_input(have_lib):
    with pytest.raises(lz.LzError):
        lz.encode(b"@r\nAC\n+\n", kind=1)            # partial FASTQ record
    with pytest.raises(lz.LzError):
        lz.encode(b"abc", min_match=3, hash_len=4)    # m < h


def test_library_exports_every_declared_symbol(have_lib):
    """Every function include/lz.h declares is exported by liblz.so."""
    import os
    import re
    from paper_2606_18900_amd import _lib
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "lz.h")).read()
    declared = set(re.findall(r"^(?:int|void|const char\*)\s+(lz_\w+)\s*\(", hdr, re.M))
    assert declared == set(_lib.EXPORTS)
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_segmented_parse_round_trip_and_thread_independence(have_lib):
    """The segmented parse (bounded memory, for inputs of many GB) writes an
    archive that the oracle decodes to the input, whose bytes do not depend on
    the thread count, and whose sources from earlier segments lie at least 32
    segments back (segments of one block here, so that rule is exercised)."""
    import oracle
    import paper_2606_18900_amd as lz
    from gen.fasta import fasta
    x = fasta(3_000_000, seed=3)
    p = dict(kind=2, block_log2=12, segment_log2=12, hash_bits=20, chain_depth=4)
    a1 = lz.encode(x, threads=1, **p)
    a8 = lz.encode(x, threads=8, **p)
    assert a1 == a8
    rc, y = oracle.decode(a1)
    assert rc == 0 and y == x
    assert len(a1) < len(x) / 2           # repeats are still found
    # segments are one block here: every dependency of block b lies 32 or
    # more blocks back (read from the archive's dependency lists)
    import numpy as np
    u64 = lambda o: int.from_bytes(a1[o:o + 8], "little")
    nb, off_ptr, off_idx = u64(32), u64(72), u64(80)
    ptr = np.frombuffer(a1, dtype=np.uint64, count=nb + 1, offset=off_ptr).astype(np.int64)
    idx = np.frombuffer(a1, dtype=np.uint32, count=int(ptr[-1]), offset=off_idx).astype(np.int64)
    owner = np.repeat(np.arange(nb), np.diff(ptr))
    assert idx.size > 0 and np.all(owner - idx >= 32)


def test_segmented_parse_rejects_bad_segment_size(have_lib):
    import paper_2606_18900_amd as lz
    with pytest.raises(Exception):
        lz.encode(b"x" * 1000, block_log2=14, segment_log2=13)   # smaller than a block
    with pytest.raises(Exception):
        lz.encode(b"x" * 1000, segment_log2=25)


SPLIT_P = dict(block_log2=10, max_level=8, min_match=16, hash_len=16, hash_bits=16, chain_depth=16,
               window_log2=0, lit_lanes=64, seq_lanes=16, prob_bits=(11, 10, 10, 10), level_penalty=8)


def test_split_container_identical_to_oracle(have_lib):
    """lz_encode_split writes the stream-separated container of the oracle's
    plain definition byte for byte (also with no records at all)."""
    import oracle.split as sp
    from gen.fastq import fastq
    x, _ = fastq(n_records=500, seed=21)
    x = bytes(x)
    assert lz.encode_split(x, **SPLIT_P) == sp.encode(x, **SPLIT_P)
    assert lz.encode_split(x, threads=3, **SPLIT_P) == sp.encode(x, **SPLIT_P)
    assert lz.encode_split(b"", **SPLIT_P) == sp.encode(b"", **SPLIT_P)


def test_split_encoder_refuses_what_the_definition_refuses(have_lib):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "split_fastq.json")))
    for text in g["rejected"]:
        with pytest.raises(lz.LzError) as e:
            lz.encode_split(text.encode(), **SPLIT_P)
        assert e.value.code == -1, text
