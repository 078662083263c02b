"""Pins for the oracle's match search: with unbounded chain depth and window the
hash-chain parse equals an exhaustive O(N^2) search (tests/ref/brute.py) on tiny
adversarial inputs, including ones that force the level cap."""
import numpy as np
import pytest

from tests.ref import brute


def _inputs():
    rng = np.random.default_rng(7)
    out = {
        "random4": rng.integers(0, 4, 1500, dtype=np.uint8).tobytes(),
        "random2": rng.integers(0, 2, 900, dtype=np.uint8).tobytes(),
        "incompressible": rng.integers(0, 256, 1200, dtype=np.uint8).tobytes(),
        "allsame": b"A" * 1000,
        "empty": b"",
        "one": b"Z",
    }
    for per in (1, 2, 3, 7, 61, 64):
        unit = rng.integers(0, 256, per, dtype=np.uint8).tobytes()
        out["period%d" % per] = (unit * (1100 // per + 1))[:1100]
    # repeats of a few motifs at random places: many inter-block sources
    motifs = [rng.integers(65, 69, 40, dtype=np.uint8).tobytes() for _ in range(5)]
    s = bytearray()
    while len(s) < 2000:
        s += motifs[int(rng.integers(0, 5))] if rng.random() < 0.6 else \
            rng.integers(65, 91, int(rng.integers(1, 30)), dtype=np.uint8).tobytes()
    out["motifs"] = bytes(s[:2000])
    from gen.fastq import fastq
    out["fastq"] = fastq(n_records=8, seed=3)[0]
    return out


INPUTS = _inputs()


def _oracle_seqs(p):
    return [(int(b), int(l), int(m), int(o)) for b, l, m, o in
            zip(p["blk"], p["ll"], p["ml"], p["of"])]


@pytest.mark.parametrize("name", sorted(INPUTS))
@pytest.mark.parametrize("bl,m,h,D,beta", [
    (6, 4, 4, 64, 0), (8, 4, 4, 64, 0), (6, 6, 4, 64, 0),
    (6, 4, 4, 4, 0), (6, 4, 4, 2, 0), (6, 4, 4, 1, 0),
    (6, 4, 4, 64, 3), (8, 5, 4, 3, 2),
])
def test_parse_equals_brute_force(orc, name, bl, m, h, D, beta):
    x = INPUTS[name]
    # 12 hash bits: collisions are frequent and must be harmless
    p = orc.parse(x, block_log2=bl, min_match=m, hash_len=h, hash_bits=12,
                  chain_depth=0, window_log2=0, max_level=D, level_penalty=beta)
    seqs, level = brute.brute_parse(x, bl, m, D, beta)
    assert _oracle_seqs(p) == seqs
    assert [int(v) for v in p["level"]] == level


def test_level_cap_is_binding(orc):
    # every block repeats the previous one: uncapped levels would climb by one
    # per block; the cap holds them at D-1
    rng = np.random.default_rng(1)
    unit = rng.integers(0, 256, 64, dtype=np.uint8).tobytes()
    x = unit * 40
    for D in (1, 2, 4, 8):
        p = orc.parse(x, block_log2=6, min_match=4, hash_len=4, hash_bits=16,
                      chain_depth=0, window_log2=0, max_level=D)
        assert int(p["level"].max()) <= D - 1
    # chain depth 1: the most recent copy (previous block) ties on length with
    # the anchor (block 0, level 0); the lower level wins, so no chain forms
    p = orc.parse(x, block_log2=6, min_match=4, hash_len=4, hash_bits=16,
                  chain_depth=1, window_log2=0, max_level=64)
    assert [int(v) for v in p["level"]] == [0] + [1] * 39


def test_parse_invariants_fastq(orc):
    """Sequences tile every block exactly, OF < write position, ML >= m except a
    final ML = 0, and each level is 1 + max level of the earlier blocks its
    sources touch (recomputed here from the parse output)."""
    from gen.fastq import fastq
    x = fastq(n_records=600, seed=9)[0]
    bl, m = 10, 16
    p = orc.parse(x, block_log2=bl, min_match=m, level_penalty=32)
    B = 1 << bl
    nb = (len(x) + B - 1) // B
    pos = {b: b * B for b in range(nb)}
    lv = [0] * nb
    last = {}
    for b, L, M, O in _oracle_seqs(p):
        pos[b] += L
        if M:
            assert M >= m and O < pos[b]
            assert x[O:O + M] == x[pos[b]:pos[b] + M] or O + M > pos[b]
            if O < b * B:
                hi = min(O + M, b * B)
                lv[b] = max(lv[b], 1 + max(lv[a] for a in range(O >> bl, ((hi - 1) >> bl) + 1)))
        pos[b] += M
        last[b] = M
    for b in range(nb):
        assert pos[b] == min(b * B + B, len(x))
    assert [int(v) for v in p["level"]] == lv
