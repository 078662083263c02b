"""Tiny pure-Python references that pin the C oracle from outside it.

* ``brute_parse``: the greedy parse by exhaustive search.  At every position it
  considers *every* earlier position whose next m bytes are equal (exactly the
  positions a match of length >= m can start from), most recent first, with no
  hashing, no chains, no anchor table.  With unbounded chain depth and window
  the hash-chain parse must produce the same sequences.
* ``rans_encode`` / ``rans_decode``: a direct rendering of rANS (Duda 2013) with
  interleaved lanes (Giesen 2014) on Python integers.
* ``fnv1a64``: FNV-1a-64 from its published constants.
"""
from __future__ import annotations

FNV_BASIS = 0xCBF29CE484222325
FNV_PRIME = 0x100000001B3


def fnv1a64(data: bytes, h: int = FNV_BASIS) -> int:
    for c in data:
        h = ((h ^ c) * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def brute_parse(x: bytes, block_log2: int, m: int, max_level: int = 64,
                level_penalty: int = 0):
    """Return (seqs, levels): seqs = list of (block, LL, ML, OF)."""
    B = 1 << block_log2
    n = len(x)
    nb = (n + B - 1) // B
    level = [0] * nb
    seqs = []
    grams: dict[bytes, list[int]] = {}
    ins = 0
    for b in range(nb):
        sb, eb = b * B, min(b * B + B, n)
        p, lit, blevel = sb, sb, 0
        while p < eb:
            while ins < p:
                if ins + m <= n:
                    grams.setdefault(x[ins:ins + m], []).append(ins)
                ins += 1
            best = None  # (score, L, lv, q)
            if p + m <= eb:
                for q in reversed(grams.get(x[p:p + m], [])):
                    cap = eb - p
                    L = 0
                    while L < cap and x[q + L] == x[p + L]:
                        L += 1
                    assert L >= m
                    if q >= sb:
                        lv = 0
                    else:
                        hi = min(q + L, sb)
                        lv = 1 + max(level[q >> block_log2:((hi - 1) >> block_log2) + 1])
                    if lv > max_level - 1:
                        continue
                    sc = L - level_penalty * lv
                    if sc < m:
                        continue
                    if best is None or sc > best[0] or (sc == best[0] and lv < best[2]):
                        best = (sc, L, lv, q)
            if best is not None:
                _, L, lv, q = best
                seqs.append((b, p - lit, L, q))
                blevel = max(blevel, lv)
                p += L
                lit = p
            else:
                p += 1
        if lit < eb:
            seqs.append((b, eb - lit, 0, 0))
        level[b] = blevel
    return seqs, level


def _cum(freq):
    c = [0]
    for f in freq:
        c.append(c[-1] + f)
    return c


def lane_runs(n: int, K: int):
    """Each lane's run of consecutive symbols: the n symbols are cut into K
    runs, the first n mod K of them one symbol longer.  Returns a list of
    (start, length) per lane."""
    runs, start = [], 0
    for k in range(K):
        ln = n // K + (1 if k < n % K else 0)
        runs.append((start, ln))
        start += ln
    assert start == n
    return runs


def decode_order(n: int, K: int):
    """(round, lane, symbol index) in the decoder's order: round by round, lanes
    ascending, a lane taking part while its run lasts."""
    runs = lane_runs(n, K)
    order = []
    for r in range(max((ln for _, ln in runs), default=0)):
        for k, (st, ln) in enumerate(runs):
            if r < ln:
                order.append((r, k, st + r))
    return order


def rans_encode(sym: bytes, freq, P: int, K: int):
    """Return (states, group_words, words_by_group) — states are the encoder's
    final states, i.e. the decoder's initial states."""
    L = 1 << 16
    c = _cum(freq)
    x = [L] * K
    order = decode_order(len(sym), K)
    emitted = {}
    for t in range(len(order) - 1, -1, -1):
        _, k, i = order[t]
        s = sym[i]
        f = freq[s]
        if x[k] >= f << (32 - P):
            emitted[t] = x[k] & 0xFFFF
            x[k] >>= 16
        x[k] = (x[k] // f) * (1 << P) + (x[k] % f) + c[s]
    G = (K + 63) // 64
    groups = [[emitted[t] for t in sorted(emitted) if order[t][1] // 64 == g] for g in range(G)]
    return x, groups


def rans_decode(states, groups, n: int, freq, P: int, K: int) -> bytes:
    L = 1 << 16
    M = 1 << P
    c = _cum(freq)
    x = list(states)
    pos = [0] * len(groups)
    out = bytearray(n)
    order = decode_order(n, K)
    rounds = {}
    for r, k, i in order:
        rounds.setdefault(r, []).append((k, i))
    for r in sorted(rounds):
        for k, i in rounds[r]:
            slot = x[k] % M
            s = next(t for t in range(256) if c[t] <= slot < c[t + 1])
            x[k] = freq[s] * (x[k] >> P) + slot - c[s]
            out[i] = s
        for k, _ in rounds[r]:
            if x[k] < L:
                g = k // 64
                x[k] = (x[k] << 16) | groups[g][pos[g]]
                pos[g] += 1
    assert all(v == L for v in x)
    assert all(pos[g] == len(groups[g]) for g in range(len(groups)))
    return bytes(out)
