"""Pins for the oracle's entropy stage (rANS, Duda 2013; lane interleaving,
Giesen 2014): round trips, an independent Python rendering, the closed-form
codelength bound, normalisation special cases and corruption detection."""
import math

import numpy as np
import pytest

from tests.ref import brute


def _freq_for(orc, sym: bytes, P: int):
    counts = np.bincount(np.frombuffer(sym, dtype=np.uint8), minlength=256)
    rc, f = orc.normalize(counts, P)
    assert rc == 0
    return f


def test_normalize_hand_examples(orc):
    # three equal counts into M = 4: floor gives 1 each, the remainder of 1
    # goes to the most frequent symbol with the lowest value
    c = np.zeros(256, np.uint64); c[[5, 9, 200]] = 1
    rc, f = orc.normalize(c, 2)
    assert rc == 0 and f[5] == 2 and f[9] == 1 and f[200] == 1 and f.sum() == 4
    # excess: 300/303*4 -> 3, three rare symbols forced to 1 -> sum 6; two units
    # are removed from the largest f > 1
    c = np.zeros(256, np.uint64); c[0] = 300; c[[1, 2, 3]] = 1
    rc, f = orc.normalize(c, 2)
    assert rc == 0 and list(f[:4]) == [1, 1, 1, 1]
    # a single symbol takes the whole range
    c = np.zeros(256, np.uint64); c[65] = 7
    rc, f = orc.normalize(c, 12)
    assert rc == 0 and f[65] == 4096 and f.sum() == 4096
    # empty histogram -> all-zero table
    rc, f = orc.normalize(np.zeros(256, np.uint64), 12)
    assert rc == 0 and f.sum() == 0
    # more symbols than slots cannot be normalised
    rc, f = orc.normalize(np.ones(256, np.uint64), 7)
    assert rc != 0


@pytest.mark.parametrize("P", [8, 10, 12])
def test_normalize_properties(orc, P):
    rng = np.random.default_rng(P)
    for _ in range(50):
        k = int(rng.integers(1, 256))
        c = np.zeros(256, np.uint64)
        idx = rng.choice(256, size=k, replace=False)
        c[idx] = rng.integers(1, 10**6, size=k) ** rng.integers(1, 3)
        rc, f = orc.normalize(c, P)
        assert rc == 0
        assert int(f.sum()) == 1 << P
        assert np.all((f > 0) == (c > 0))


def test_lanes_rule(orc):
    assert orc.rans_lanes(0, 64) == 1
    assert orc.rans_lanes(15, 64) == 1
    assert orc.rans_lanes(32, 64) == 2
    assert orc.rans_lanes(16000, 256) == 256
    assert orc.rans_lanes(16000, 100) == 100
    assert orc.rans_lanes(1000, 256) == 32
    # short streams: 4 symbols per lane
    assert orc.rans_lanes(3, 64, 4) == 1
    assert orc.rans_lanes(120, 64, 4) == 16
    assert orc.rans_lanes(4100, 64, 4) == 64


def test_lane_runs_hand_example():
    # 5 symbols over 2 lanes: lane 0 holds symbols 0..2, lane 1 symbols 3..4;
    # the decoder takes them round by round, lanes ascending
    assert brute.lane_runs(5, 2) == [(0, 3), (3, 2)]
    assert brute.decode_order(5, 2) == [(0, 0, 0), (0, 1, 3), (1, 0, 1), (1, 1, 4), (2, 0, 2)]
    # fewer symbols than lanes: the tail lanes hold nothing
    assert brute.lane_runs(2, 4) == [(0, 1), (1, 1), (2, 0), (2, 0)]


def test_single_lane_is_plain_rans(orc):
    """With one lane the body is the textbook rANS coder: a single state,
    words in the order the decoder reads them (Duda 2013)."""
    sym = bytes([3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5] * 20)
    freq = _freq_for(orc, sym, 8)
    rc, body, nw = orc.rans_encode(sym, freq, 8, 1)
    assert rc == 0
    c = [0]
    for v in freq:
        c.append(c[-1] + int(v))
    x = 1 << 16
    words = []
    for s in reversed(sym):
        f = int(freq[s])
        if x >= f << 24:
            words.append(x & 0xFFFF)
            x >>= 16
        x = (x // f) * 256 + x % f + c[s]
    words.reverse()
    ref = x.to_bytes(4, "little") + len(words).to_bytes(4, "little")
    ref += b"".join(w.to_bytes(2, "little") for w in words)
    assert body == ref and nw == len(words)


def _streams():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 63, 64, 65, 129, 1000, 4097):
        out.append(("uni%d" % n, rng.integers(0, 256, n, dtype=np.uint8).tobytes()))
    skew = rng.geometric(0.3, 3000).clip(0, 255).astype(np.uint8)
    skew[::997] = 255                     # rare symbols that normalise to f = 1
    out.append(("skew", skew.tobytes()))
    out.append(("two", (rng.random(2000) < 0.999).astype(np.uint8).tobytes()))
    return out


@pytest.mark.parametrize("P", [8, 10, 12])
@pytest.mark.parametrize("K", [1, 8, 64, 100, 256])
def test_roundtrip_and_reference(orc, P, K):
    for name, sym in _streams():
        freq = _freq_for(orc, sym, P)
        rc, body, nw = orc.rans_encode(sym, freq, P, K)
        assert rc == 0, name
        G = (K + 63) // 64
        assert len(body) == 4 * K + 4 * G + 2 * nw
        rc, out = orc.rans_decode(body, len(sym), nw, freq, P, K)
        assert rc == 0 and out == sym, name
        if len(sym) <= 1000:
            states, groups = brute.rans_encode(sym, [int(v) for v in freq], P, K)
            ref = b"".join(int(s).to_bytes(4, "little") for s in states)
            ref += b"".join(len(g).to_bytes(4, "little") for g in groups)
            ref += b"".join(int(w).to_bytes(2, "little") for g in groups for w in g)
            assert body == ref, name
            assert brute.rans_decode(states, groups, len(sym), [int(v) for v in freq], P, K) == sym


@pytest.mark.parametrize("P", [8, 12])
def test_codelength_bound(orc, P):
    """16 * n_words <= sum_i log2(M / f_{s_i}) + n log2(1 + 2^(P-16)): each step
    grows log2(x) by at most log2(M/f) + log2(1 + f/x) and f/x <= 2^(P-16)
    after renormalisation; the final state of every lane is >= 2^16."""
    rng = np.random.default_rng(5)
    for K in (1, 64, 256):
        sym = rng.geometric(0.15, 50000).clip(0, 255).astype(np.uint8).tobytes()
        freq = _freq_for(orc, sym, P)
        rc, body, nw = orc.rans_encode(sym, freq, P, K)
        assert rc == 0
        M = 1 << P
        info = sum(math.log2(M / int(freq[s])) for s in sym)
        slack = len(sym) * math.log2(1 + 2.0 ** (P - 16))
        assert 16 * nw <= info + slack + 1e-6
        # and the code is close to the empirical entropy (lanes cost <= 32 bits each)
        assert 16 * nw + 32 * K <= info + slack + 32 * K


def test_corruption_detected(orc):
    rng = np.random.default_rng(3)
    sym = rng.geometric(0.2, 5000).clip(0, 255).astype(np.uint8).tobytes()
    freq = _freq_for(orc, sym, 12)
    rc, body, nw = orc.rans_encode(sym, freq, 12, 64)
    assert rc == 0
    # truncated body: size check
    rc, _ = orc.rans_decode(body[:-2], len(sym), nw, freq, 12, 64)
    assert rc == orc.ECORRUPT
    # a flipped initial state or word: the end-state check fires (or, if the
    # damage cancels, the symbols differ)
    for pos in (0, 4 * 64 + 4 + 10, len(body) - 1):
        bad = bytearray(body)
        bad[pos] ^= 0x5A
        rc, out = orc.rans_decode(bytes(bad), len(sym), nw, freq, 12, 64)
        assert rc == orc.ECORRUPT or out != sym
    # state below 2^16
    bad = bytearray(body); bad[0:4] = (5).to_bytes(4, "little")
    rc, _ = orc.rans_decode(bytes(bad), len(sym), nw, freq, 12, 64)
    assert rc == orc.ECORRUPT
