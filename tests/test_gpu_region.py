"""GPU parity for FASTA coordinate access (lz_decode_region): bases of a
sequence by (name, start, end), compared with the oracle's plain definition
(sequence lines joined, sliced) on regions inside one line, across line ends,
at both ends of a sequence, and the error cases."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def genome(orc):
    import paper_2606_18900_amd as lz
    from gen.fasta import fasta
    x = fasta(4_000_000, seed=3)
    a = orc.encode(x, kind=2, level_penalty=32)
    return x, lz.Archive(a), lz.fasta_index(x), orc.fasta_sequences(x)


def test_regions_match_plain_definition(genome, orc):
    from paper_2606_18900_amd import _lib
    x, arc, idx, seqs = genome
    rng = np.random.default_rng(12)
    cases = []
    for sq in idx:
        L = int(sq.length)
        cases += [(sq, 0, min(L, 10)), (sq, max(0, L - 7), L), (sq, 59, 61), (sq, 0, min(L, 60 * 40 + 3))]
        for _ in range(4):
            s = int(rng.integers(0, L))
            cases.append((sq, s, min(L, s + int(rng.integers(1, 50_000)))))
    for sq, s, e in cases:
        got = arc.decode_region(sq, s, e)
        torch.cuda.synchronize()
        arc.sync_status()
        assert got.cpu().numpy().tobytes() == seqs[sq.name.decode()][0][s:e], (sq.name, s, e)
    sq = idx[3]
    assert arc.decode_region(sq, 5, 5).numel() == 0
    with pytest.raises(_lib.LzError) as ei:
        arc.decode_region(sq, 0, int(sq.length) + 1)
    assert ei.value.code == _lib.LZ_ERANGE
    bad = _lib.FastaSeq()
    bad.offset, bad.length, bad.line_bases, bad.line_bytes = sq.offset, sq.length, 0, 0
    with pytest.raises(_lib.LzError) as ei:
        arc.decode_region(bad, 0, 10)
    assert ei.value.code == _lib.LZ_ENOINDEX
