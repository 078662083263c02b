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
