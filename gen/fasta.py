"""Seeded synthetic genome FASTA generator (stand-in for the paper's 5 GB / 50 GB
"genome" inputs of Table 3 and the 50 GB range-decode experiment, which are not
available here).

File layout: 24 records ``>chr1`` .. ``>chr22``, ``>chrX``, ``>chrY``; sequence
lengths proportional to (25 - i) for the i-th record, the last one sized so the
file is exactly ``total_bytes`` long; 60 bases per line, every line (also the
last, partial one) ends in ``\\n``; uppercase ACGTN.

Sequence content, built chunk by chunk (each chunk has its own RNG stream,
derived from (seed, record, chunk), so chunks can be built independently):
* background: i.i.d. A/T 0.295 each, G/C 0.205 each (GC 41 %);
* features separated by background runs (geometric, mean 1972 bp); a feature is
  an interspersed-repeat copy with probability 0.9 or a tandem array with
  probability 0.1, which gives about 45 % repeat and 3 % tandem coverage;
* repeat copy: a whole element of a 500-element library (lengths log-uniform in
  [300, 6000] bp, element chosen with Zipf s = 1), forward strand, each base
  substituted with probability d ~ U[0.05, 0.20];
* tandem array: unit length log-uniform in [2, 200], array length log-uniform in
  [50, 5000], 1 % substitutions;
* N runs: min(10000, len/20) at both record ends and one run of 0.5 % of the
  record length at a random interior position.
Nothing here touches the codec.
"""
from __future__ import annotations

import os
import numpy as np

LINE = 60
CHUNK = LINE * (1 << 18)          # bases per generation chunk (15.7 Mbp)
NAMES = [f"chr{i}" for i in range(1, 23)] + ["chrX", "chrY"]
_BG_P = np.array([0.295, 0.205, 0.205, 0.295])
_BG_CDF = np.cumsum(_BG_P)
_ACGTN = np.frombuffer(b"ACGTN", dtype=np.uint8)


def _rec_size(name: str, L: int) -> int:
    return 1 + len(name) + 1 + L + -(-L // LINE)


def layout(total_bytes: int) -> list[tuple[str, int, int]]:
    """[(name, seq_len, file_offset)] with the file exactly total_bytes long."""
    hdr = sum(len(n) + 2 for n in NAMES)
    budget = total_bytes - hdr
    if budget < 24 * 2:
        raise ValueError("total_bytes too small for 24 records")
    w = np.array([25 - i for i in range(1, 25)], dtype=np.float64)
    seq_budget = budget * LINE // (LINE + 1)
    lens = [max(1, int(seq_budget * wi / w.sum())) for wi in w[:-1]]
    while True:
        used = sum(_rec_size(n, L) for n, L in zip(NAMES[:-1], lens))
        rem = total_bytes - used - (len(NAMES[-1]) + 2)
        L = rem * LINE // (LINE + 1)
        while L + -(-L // LINE) < rem:
            L += 1
        if L >= 1 and L + -(-L // LINE) == rem:
            break
        lens[-1] += 1
    lens.append(L)
    out, off = [], 0
    for n, L in zip(NAMES, lens):
        out.append((n, L, off))
        off += _rec_size(n, L)
    assert off == total_bytes
    return out


def _library(seed: int) -> list[np.ndarray]:
    rng = np.random.default_rng([seed, 7777])
    lens = np.exp(rng.uniform(np.log(300), np.log(6000), size=500)).astype(np.int64)
    return [np.searchsorted(_BG_CDF, rng.random(int(L)), side="right").astype(np.uint8)
            for L in lens]


_ZIPF = 1.0 / np.arange(1, 501)
_ZIPF_CDF = np.cumsum(_ZIPF / _ZIPF.sum())


def _subst(rng, codes: np.ndarray, p: float) -> None:
    m = rng.random(codes.shape[0]) < p
    k = int(m.sum())
    if k:
        codes[m] = (codes[m] + rng.integers(1, 4, size=k, dtype=np.uint8)) % 4


def _chunk_codes(seed: int, rec: int, chunk: int, n: int, lib) -> np.ndarray:
    rng = np.random.default_rng([seed, rec, chunk])
    out = np.searchsorted(_BG_CDF, rng.random(n), side="right").astype(np.uint8)
    p = int(rng.geometric(1.0 / 1972.0)) // 2      # first feature starts mid-run
    while p < n:
        if rng.random() < 0.9:
            e = int(np.searchsorted(_ZIPF_CDF, rng.random(), side="right"))
            seg = lib[min(e, 499)].copy()
            _subst(rng, seg, rng.uniform(0.05, 0.20))
        else:
            u = int(np.exp(rng.uniform(np.log(2), np.log(200))))
            a = int(np.exp(rng.uniform(np.log(50), np.log(5000))))
            unit = np.searchsorted(_BG_CDF, rng.random(u), side="right").astype(np.uint8)
            seg = np.resize(unit, a)
            _subst(rng, seg, 0.01)
        q = min(n, p + seg.shape[0])
        out[p:q] = seg[: q - p]
        p = q + int(rng.geometric(1.0 / 1972.0))
    return out


def _n_runs(seed: int, rec: int, L: int) -> list[tuple[int, int]]:
    rng = np.random.default_rng([seed, rec, 99991])
    e = min(10000, L // 20)
    mid = (5 * L) // 1000
    s = int(rng.integers(0, max(1, L - mid)))
    return [(0, e), (L - e, L), (s, s + mid)]


def _render_chunk(seed: int, rec: int, L: int, chunk: int, lib) -> np.ndarray:
    b0 = chunk * CHUNK
    n = min(CHUNK, L - b0)
    codes = _chunk_codes(seed, rec, chunk, n, lib)
    for s, e in _n_runs(seed, rec, L):
        s2, e2 = max(s, b0), min(e, b0 + n)
        if s2 < e2:
            codes[s2 - b0:e2 - b0] = 4
    bases = _ACGTN[codes]
    full = n // LINE
    tail = n - full * LINE
    out = np.empty(full * (LINE + 1) + (tail + 1 if tail else 0), dtype=np.uint8)
    body = out[: full * (LINE + 1)].reshape(full, LINE + 1)
    body[:, :LINE] = bases[: full * LINE].reshape(full, LINE)
    body[:, LINE] = 10
    if tail:
        out[full * (LINE + 1):-1] = bases[full * LINE:]
        out[-1] = 10
    return out


def _jobs(total_bytes: int):
    for rec, (name, L, off) in enumerate(layout(total_bytes)):
        hdr = (">" + name + "\n").encode()
        yield ("hdr", off, hdr)
        base_off = off + len(hdr)
        for c in range(-(-L // CHUNK)):
            yield ("seq", base_off + c * (CHUNK + CHUNK // LINE), (rec, L, c))


def _work(args):
    seed, path, off, rec, L, c = args
    lib = _library(seed)
    buf = _render_chunk(seed, rec, L, c, lib)
    with open(path, "r+b") as f:
        f.seek(off)
        f.write(buf.tobytes())
    return len(buf)


def fasta(total_bytes: int, seed: int = 3, out_path: str | None = None,
          workers: int = 1) -> bytes | None:
    """Build the genome; return the bytes, or write them to out_path (chunks in
    parallel with `workers` processes) and return None."""
    if out_path is None:
        lib = _library(seed)
        out = np.empty(total_bytes, dtype=np.uint8)
        for kind, off, payload in _jobs(total_bytes):
            if kind == "hdr":
                out[off:off + len(payload)] = np.frombuffer(payload, dtype=np.uint8)
            else:
                rec, L, c = payload
                buf = _render_chunk(seed, rec, L, c, lib)
                out[off:off + buf.shape[0]] = buf
        return out.tobytes()
    with open(out_path, "wb") as f:
        f.truncate(total_bytes)
    tasks = []
    with open(out_path, "r+b") as f:
        for kind, off, payload in _jobs(total_bytes):
            if kind == "hdr":
                f.seek(off)
                f.write(payload)
            else:
                tasks.append((seed, out_path, off) + tuple(payload))
    if workers <= 1:
        for t in tasks:
            _work(t)
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_work, tasks):
                pass
    assert os.path.getsize(out_path) == total_bytes
    return None
