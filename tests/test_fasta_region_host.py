"""Coordinate access to FASTA (chr:pos), host side: the oracle's plain
definition is pinned by a hand-written file and by the generator's own layout
(sequence lengths and offsets computed from the record sizes, not by parsing),
and the product's .fai-style index agrees with both."""
import numpy as np
import pytest


HAND = b">chrA desc\nACGTA\nCCGTT\nGG\n>chrB\nNNNNN\nA\n"


def test_oracle_region_hand_example(orc):
    seqs = orc.fasta_sequences(HAND)
    assert seqs["chrA"] == (b"ACGTACCGTTGG", 11)
    assert seqs["chrB"] == (b"NNNNNA", HAND.index(b"NNNNN"))
    assert orc.fasta_region(HAND, "chrA", 3, 8) == b"TACCG"      # crosses a line end
    assert orc.fasta_region(HAND, "chrB", 0, 6) == b"NNNNNA"
    assert orc.fasta_region(HAND, "chrA", 4, 4) == b""


def test_oracle_region_matches_generator_layout(orc):
    from gen.fasta import fasta, layout
    N = 2_000_000
    x = fasta(N, seed=3)
    seqs = orc.fasta_sequences(x)
    lay = layout(N)
    assert list(seqs) == [n for n, _, _ in lay]
    for name, L, off in lay:
        s, first = seqs[name]
        assert len(s) == L and first == off + len(name) + 2
        assert set(s) <= set(b"ACGTN")


def test_product_index_agrees(orc):
    import paper_2606_18900_amd as lz
    from gen.fasta import fasta
    for text in (HAND, fasta(3_000_000, seed=3)):
        idx = lz.fasta_index(text)
        seqs = orc.fasta_sequences(text)
        assert [s.name.decode() for s in idx] == list(seqs)
        for s in idx:
            seq, first = seqs[s.name.decode()]
            assert s.offset == first and s.length == len(seq)
    idx = lz.fasta_index(HAND)
    assert (idx[0].line_bases, idx[0].line_bytes) == (5, 6)
    uneven = lz.fasta_index(b">x\nACG\nA\nACG\n")
    assert uneven[0].line_bases == 0 and uneven[0].length == 7
    with pytest.raises(Exception):
        lz.fasta_index(b"ACGT\n")
