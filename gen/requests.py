"""Seeded request streams for random-access workloads (no codec arithmetic).

* ``batched_lookups``: the batched random-access mix — single-read lookups
  (read ids half uniform, half bounded Zipf s = 1.1 over ranks mapped through a
  seeded permutation) and byte ranges starting at a record start with lengths
  log-uniform in [4 KiB, 1 MiB], clipped to the file.
* ``poisson_trace``: an open-loop Poisson arrival trace for the served loop —
  90 % single reads, 9 % ranges of 64 KiB..4 MiB (log-uniform), 1 % ranges of
  1 GiB; ranges go to either of two archives with probability 1/2.

A request is (kind, a, b): kind 0 = read (a = read id, b = 0), kind 1 = byte
range (a = offset, b = length).  ``archive`` selects the target archive.
"""
from __future__ import annotations

import numpy as np

READ, RANGE = 0, 1


def _zipf_ranks(rng, n_items: int, k: int, s: float) -> np.ndarray:
    # bounded Zipf over ranks 1..n_items by inverse CDF on a float64 table
    ranks = np.arange(1, n_items + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-s))
    cdf /= cdf[-1]
    return np.searchsorted(cdf, rng.random(k), side="right").clip(0, n_items - 1)


def read_ids(rng, n_reads: int, k: int) -> np.ndarray:
    """Half uniform, half Zipf(1.1) through a seeded permutation."""
    perm = rng.permutation(n_reads)
    uni = rng.integers(0, n_reads, size=k)
    zipf = perm[_zipf_ranks(rng, n_reads, k, 1.1)]
    pick = rng.random(k) < 0.5
    return np.where(pick, uni, zipf).astype(np.int64)


def batched_lookups(n_requests: int, record_starts: np.ndarray, total_len: int,
                    seed: int = 4, range_frac: float = 0.10):
    """Return int64 arrays (kind, a, b) of length n_requests."""
    rng = np.random.default_rng(seed)
    n_reads = record_starts.shape[0] - 1
    ids = read_ids(rng, n_reads, n_requests)
    is_range = rng.random(n_requests) < range_frac
    lens = np.exp(rng.uniform(np.log(4096), np.log(1 << 20), size=n_requests)).astype(np.int64)
    starts = record_starts[ids].astype(np.int64)
    lens = np.minimum(lens, total_len - starts)
    kind = np.where(is_range, RANGE, READ).astype(np.int64)
    a = np.where(is_range, starts, ids).astype(np.int64)
    b = np.where(is_range, lens, 0).astype(np.int64)
    return kind, a, b


def poisson_trace(rate: float, duration_s: float, fastq_starts: np.ndarray,
                  fastq_len: int, genome_len: int, seed: int = 5,
                  big_range: int = 1 << 30):
    """Return a dict of arrays: t (arrival seconds), archive (0 FASTQ, 1 genome),
    kind, a, b."""
    rng = np.random.default_rng([seed, int(rate)])
    n = int(rng.poisson(rate * duration_s))
    t = np.sort(rng.uniform(0.0, duration_s, size=n))
    u = rng.random(n)
    kind = np.where(u < 0.90, READ, RANGE).astype(np.int64)
    big = u >= 0.99
    arch = np.where(kind == READ, 0, (rng.random(n) < 0.5).astype(np.int64))
    n_reads = fastq_starts.shape[0] - 1
    ids = read_ids(rng, n_reads, n)
    rl = np.exp(rng.uniform(np.log(64 << 10), np.log(4 << 20), size=n)).astype(np.int64)
    N = np.where(arch == 0, fastq_len, genome_len)
    rl = np.where(big, big_range, rl)
    rl = np.minimum(rl, N)
    off = np.floor(rng.random(n) * (N - rl + 1)).astype(np.int64)
    a = np.where(kind == READ, ids, off)
    b = np.where(kind == READ, 0, rl)
    return {"t": t, "archive": arch, "kind": kind, "a": a.astype(np.int64),
            "b": b.astype(np.int64)}
