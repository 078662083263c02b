"""Pins of the encoder's source rebasing (orc_rebase; the format leaves the
choice among equal source positions free): every rebased match still reads
bytes equal to its destination, never moves forward, leaves no window that a
further step would move, keeps the block's dependencies, and shortens the
in-block copy chains of a FASTQ file.  Checked by brute force in Python."""
import numpy as np
import pytest

import oracle
from gen.fastq import fastq

P = dict(kind=1, block_log2=12, max_level=64, min_match=16, hash_len=16, hash_bits=18, chain_depth=16,
         level_penalty=32)


@pytest.fixture(scope="module")
def parsed():
    x, _ = fastq(n_records=900, seed=41)
    x = bytes(x)
    r = oracle.parse(x, **{k: v for k, v in P.items() if k != "kind"})
    return x, r, oracle.rebase(r, P["block_log2"])


def _matches(r, of, B):
    """Per block: list of (sequence index, destination, length, source)."""
    out = {}
    pos_blk = {}
    for q in range(len(r["blk"])):
        b = int(r["blk"][q])
        pos = pos_blk.get(b, b * B) + int(r["ll"][q])
        M = int(r["ml"][q])
        if M:
            out.setdefault(b, []).append((q, pos, M, int(of[q])))
        pos_blk[b] = pos + M
    return out


def _depth(ms):
    """In-block dependency depth: a match waits for every earlier match of the
    block whose destination meets its source window [o, o + min(p - o, M))."""
    d = []
    for a, (_, p, M, o) in enumerate(ms):
        w0, w1 = o, o + min(p - o, M)
        k = 0
        for c in range(a):
            _, pc, Mc, _ = ms[c]
            if pc < w1 and pc + Mc > w0:
                k = max(k, d[c])
        d.append(k + 1)
    return max(d) if d else 0


def test_rebased_sources_read_equal_bytes(parsed):
    x, r, of2 = parsed
    B = 1 << P["block_log2"]
    before = _matches(r, r["of"], B)
    moved = 0
    for b, ms in _matches(r, of2, B).items():
        for (q, p, M, o2), (_, _, _, o1) in zip(ms, before[b]):
            assert o2 <= o1
            if o2 != o1:
                moved += 1
                assert p - o1 >= M                    # only non-overlapping matches move
                assert x[o2:o2 + M] == x[p:p + M]
    assert moved > 0


def test_rebasing_is_a_fixed_point(parsed):
    x, r, of2 = parsed
    B = 1 << P["block_log2"]
    for b, ms in _matches(r, of2, B).items():
        for a, (_, p, M, o) in enumerate(ms):
            if p - o < M:
                continue
            for c in range(a):
                _, pc, Mc, oc = ms[c]
                assert not (pc <= o and o + M <= pc + Mc and pc - oc >= Mc), (b, a, c)


def test_dependencies_kept_and_chains_shorter(parsed):
    x, r, of2 = parsed
    B = 1 << P["block_log2"]
    d0 = d1 = 0
    before = _matches(r, r["of"], B)
    for b, ms in _matches(r, of2, B).items():
        def touched(mlist):
            s = set()
            for _, p, M, o in mlist:
                for blk in range(o // B, (o + M - 1) // B + 1):
                    if blk != b:
                        s.add(blk)
            return s
        assert touched(ms) <= touched(before[b])
        d0 += _depth(before[b])
        d1 += _depth(ms)
    assert d1 < d0


def test_encoded_archive_round_trip(parsed):
    x, _, _ = parsed
    a = oracle.encode(x, **P)
    rc, y = oracle.decode(a)
    assert rc == 0 and y == x
