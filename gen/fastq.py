"""Seeded synthetic FASTQ generator.

Stand-in for the paper's sequencing inputs (NA12878 / ERR194147 FASTQ, Table 2),
which are not available here.  The shape follows the paper's workload: 4-line
Illumina-style records with 150 bp reads and Phred+33 qualities.  Nothing in this
module touches the codec; it only produces bytes and the record starts.

Record r (0-based) of a file with nominal record count n:

    @SYN:<run>:<lane>:<tile>:<x>:<y>\\n
    <150 bases>\\n
    +\\n
    <150 qualities>\\n

* run: 4 digits, fixed per file, drawn from the seed.
* lane = 1 + floor(8 r / n); tile = 1101 + (floor(r/4000) mod 16) + 100 (floor(r/64000) mod 2).
* x, y uniform in [1000, 32767].
* Bases i.i.d. uniform over ACGT, each replaced by N with probability 0.001.
  With probability 0.02 a read (r >= 1) instead copies the bases of a uniformly
  chosen earlier read, substituting each base with probability 0.01 by one of
  the other three letters.
* Qualities: first-order Markov chain over Q2..Q40.  q0 ~ U{34..40};
  q[j+1] = clip(q[j] + floor(0.25 (mu_j - q[j]) + 0.5) + eta_j, 2, 40) with
  eta_j ~ U{-2..2} and mu_j = 38 - 14 (j/149)^2; with probability 0.002 per
  position the read drops to Q2 and stays there to its end.
"""
from __future__ import annotations

import numpy as np

READ_LEN = 150
_ACGT = np.frombuffer(b"ACGTN", dtype=np.uint8)
_FIXED_TAIL = READ_LEN + 1 + 2 + READ_LEN + 1  # bases\n +\n quals\n


def _digits(v: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Right-aligned 5-digit ASCII rendering and the digit count (4 or 5)."""
    v = v.astype(np.int64)
    nd = np.where(v >= 10000, 5, 4).astype(np.int64)
    d = np.empty((v.shape[0], 5), dtype=np.uint8)
    t = v.copy()
    for k in range(4, -1, -1):
        d[:, k] = (t % 10) + 48
        t //= 10
    return d, nd


def _bases(rng: np.random.Generator, n: int) -> np.ndarray:
    codes = rng.integers(0, 4, size=(n, READ_LEN), dtype=np.uint8)
    nmask = rng.random((n, READ_LEN)) < 0.001
    codes[nmask] = 4
    dup = rng.random(n) < 0.02
    dup[0] = False
    rows = np.flatnonzero(dup)
    src = np.floor(rng.random(rows.shape[0]) * rows).astype(np.int64)
    submask = rng.random((rows.shape[0], READ_LEN)) < 0.01
    suboff = rng.integers(1, 4, size=(rows.shape[0], READ_LEN), dtype=np.uint8)
    for k in range(rows.shape[0]):          # increasing r, so sources are final
        r = rows[k]
        row = codes[src[k]].copy()
        m = submask[k]
        if m.any():
            c = row[m]
            off = suboff[k][m]
            row[m] = np.where(c < 4, (c + off) % 4, off - 1)
        codes[r] = row
    return _ACGT[codes]


def _quals(rng: np.random.Generator, n: int) -> np.ndarray:
    q = np.empty((n, READ_LEN), dtype=np.int16)
    cur = rng.integers(34, 41, size=n).astype(np.int16)
    eta = rng.integers(-2, 3, size=(n, READ_LEN - 1)).astype(np.int16)
    drop = rng.random((n, READ_LEN)) < 0.002
    dropped = drop[:, 0].copy()
    cur[dropped] = 2
    q[:, 0] = cur
    for j in range(READ_LEN - 1):
        mu = 38.0 - 14.0 * (j / 149.0) ** 2
        step = np.floor(0.25 * (mu - cur) + 0.5).astype(np.int16)
        cur = np.clip(cur + step + eta[:, j], 2, 40).astype(np.int16)
        dropped |= drop[:, j + 1]
        cur[dropped] = 2
        q[:, j + 1] = cur
    return (q + 33).astype(np.uint8)


def fastq(n_records: int | None = None, max_bytes: int | None = None,
          seed: int = 1) -> tuple[bytes, np.ndarray]:
    """Return (data, starts): the FASTQ bytes and the u64 start of every record
    followed by len(data).  Give n_records, or max_bytes to keep the longest
    whole-record prefix of a nominal ceil(max_bytes/330)-record file."""
    if (n_records is None) == (max_bytes is None):
        raise ValueError("give exactly one of n_records, max_bytes")
    n = n_records if n_records is not None else -(-max_bytes // 330)
    if n <= 0:
        return b"", np.zeros(1, dtype=np.uint64)
    rng = np.random.default_rng(seed)
    run = int(rng.integers(1000, 10000))
    x = rng.integers(1000, 32768, size=n)
    y = rng.integers(1000, 32768, size=n)
    bases = _bases(rng, n)
    quals = _quals(rng, n)

    r = np.arange(n, dtype=np.int64)
    lane = 1 + (8 * r) // n
    tile = 1101 + (r // 4000) % 16 + 100 * ((r // 64000) % 2)
    xd, xn = _digits(x)
    yd, yn = _digits(y)
    hdr_len = 17 + xn + 1 + yn + 1
    rec_len = hdr_len + _FIXED_TAIL
    starts = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(rec_len, out=starts[1:])
    if max_bytes is not None:
        keep = int(np.searchsorted(starts, max_bytes, side="right")) - 1
        n_keep = keep
    else:
        n_keep = n
    total = int(starts[n_keep])
    out = np.empty(total, dtype=np.uint8)

    CH = 1 << 16
    rund = np.frombuffer(b"%04d" % run, dtype=np.uint8)
    for c0 in range(0, n_keep, CH):
        c1 = min(n_keep, c0 + CH)
        m = c1 - c0
        s = starts[c0:c1]
        pre = np.empty((m, 17), dtype=np.uint8)
        pre[:, 0:5] = np.frombuffer(b"@SYN:", dtype=np.uint8)
        pre[:, 5:9] = rund
        pre[:, 9] = 58
        pre[:, 10] = 48 + lane[c0:c1]
        pre[:, 11] = 58
        t = tile[c0:c1]
        for k in range(4):
            pre[:, 12 + k] = 48 + (t // 10 ** (3 - k)) % 10
        pre[:, 16] = 58
        out[s[:, None] + np.arange(17)] = pre
        # x digits (left-aligned), ':', y digits, '\n'
        xo = s + 17
        cols = np.arange(5)
        mask = cols[None, :] < xn[c0:c1, None]
        src = np.where(xn[c0:c1, None] == 5, cols[None, :], cols[None, :] + 1)
        xv = np.take_along_axis(xd[c0:c1], np.minimum(src, 4), axis=1)
        idx = xo[:, None] + cols[None, :]
        out[idx[mask]] = xv[mask]
        yo = xo + xn[c0:c1] + 1
        out[yo - 1] = 58
        mask = cols[None, :] < yn[c0:c1, None]
        src = np.where(yn[c0:c1, None] == 5, cols[None, :], cols[None, :] + 1)
        yv = np.take_along_axis(yd[c0:c1], np.minimum(src, 4), axis=1)
        idx = yo[:, None] + cols[None, :]
        out[idx[mask]] = yv[mask]
        bo = yo + yn[c0:c1] + 1
        out[bo - 1] = 10
        out[bo[:, None] + np.arange(READ_LEN)] = bases[c0:c1]
        p = bo + READ_LEN
        out[p] = 10
        out[p + 1] = 43
        out[p + 2] = 10
        qo = p + 3
        out[qo[:, None] + np.arange(READ_LEN)] = quals[c0:c1]
        out[qo + READ_LEN] = 10
    st = starts[: n_keep + 1].astype(np.uint64)
    return out.tobytes(), st
