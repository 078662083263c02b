"""Pins for the oracle's container, decoder, validator, read index and range
decode: the plain definition decode(encode(x)) == x on every workload shape,
invariants recomputed from the bytes, corruptions rejected, and the paper's
unit arithmetic."""
import json
import os

import numpy as np
import pytest

from tests.ref import brute

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
FASTQ_PARAMS = dict(kind=1, level_penalty=32)


@pytest.fixture(scope="module")
def fq(orc):
    from gen.fastq import fastq
    x, starts = fastq(n_records=1500, seed=21)
    return x, starts, orc.encode(x, **FASTQ_PARAMS)


def test_paper_unit_arithmetic(orc):
    B = GOLD["block_bytes"]["value"]
    assert B == 1 << 14
    N = GOLD["scale_total_bytes"]["value"]
    assert -(-N // B) == GOLD["scale_blocks"]["value"]
    assert round(N / 1e9 / (GOLD["scale_ms"]["value"] / 1e3), 1) == GOLD["scale_gbps"]["value"]
    assert GOLD["index_reads"]["value"] * GOLD["index_bytes_per_read"]["value"] == GOLD["index_bytes"]["value"]
    assert round(5e9 / 1e9 / (GOLD["table3_full_ms"]["value"] / 1e3)) == GOLD["table3_full_gbps"]["value"]
    # the oracle's archives use that block size and count
    for n in (1, B - 1, B, B + 1, 3 * B + 7):
        x = bytes(np.random.default_rng(n).integers(0, 4, n, dtype=np.uint8))
        i = orc.info(orc.encode(x))
        assert i.n == n and i.n_blocks == -(-n // B) and i.block_log2 == 14


@pytest.mark.parametrize("shape", ["empty", "one", "B", "B+1", "random", "allsame", "fasta"])
def test_roundtrip(orc, shape):
    rng = np.random.default_rng(2)
    B = 1 << 14
    x = {"empty": b"", "one": b"x", "B": rng.integers(0, 256, B, dtype=np.uint8).tobytes(),
         "B+1": rng.integers(0, 3, B + 1, dtype=np.uint8).tobytes(),
         "random": rng.integers(0, 256, 70000, dtype=np.uint8).tobytes(),
         "allsame": b"N" * 100000}.get(shape)
    kind = 0
    if shape == "fasta":
        from gen.fasta import fasta
        x, kind = fasta(3_000_000, seed=3), 2
    a = orc.encode(x, kind=kind, level_penalty=32)
    assert orc.validate(a) == 0
    rc, out = orc.decode(a)
    assert rc == 0 and out == x
    i = orc.info(a)
    assert i.source_fnv == _tree(x)


def _tree(x, B=1 << 14):
    h = brute.FNV_BASIS
    for b in range(0, len(x), B):
        h = brute.fnv1a64(brute.fnv1a64(x[b:b + B]).to_bytes(8, "little"), h)
    return h


def test_fnv_published_vectors(orc):
    # FNV-1a-64 reference values (published test vectors of the FNV authors)
    assert orc.fnv1a64(b"") == 0xCBF29CE484222325
    assert orc.fnv1a64(b"a") == 0xAF63DC4C8601EC8C
    assert orc.fnv1a64(b"foobar") == 0x85944171F73967E8
    assert brute.fnv1a64(b"foobar") == 0x85944171F73967E8


@pytest.mark.parametrize("lanes", [1, 16, 64, 200, 256])
def test_roundtrip_lane_counts(orc, fq, lanes):
    x, _, _ = fq
    a = orc.encode(x, lit_lanes=lanes, seq_lanes=min(lanes, 64), **FASTQ_PARAMS)
    rc, out = orc.decode(a)
    assert rc == 0 and out == x


def test_fastq_roundtrip_and_index(orc, fq):
    x, starts, a = fq
    rc, out = orc.decode(a)
    assert rc == 0 and out == x
    i = orc.info(a)
    assert i.n_reads == len(starts) - 1 and i.kind == 1
    # the index section is exactly 8 bytes per read (+ the end sentinel)
    off = int.from_bytes(a[96:104], "little")
    idx = np.frombuffer(a[off:off + 8 * (i.n_reads + 1)], dtype=np.uint64)
    assert len(a) - off == 8 * (i.n_reads + 1)
    assert np.array_equal(idx, starts)
    # every read id maps to its block and byte: line 4r starts there
    lines = x.split(b"\n")
    for r in (0, 1, 777, i.n_reads - 1):
        s = int(idx[r])
        assert x[s:s + 1] == b"@"
        assert x[s:int(idx[r + 1])] == b"\n".join(lines[4 * r:4 * r + 4]) + b"\n"
        assert (s >> 14, s & 16383) == divmod(s, 16384)
    assert i.max_record_len == int(np.diff(starts).max())


def test_read_index_counts_lines_not_at_signs(orc):
    # qualities that start with '@' (Q31) must not split records
    rec = b"@r1\nACGT\n+\n@@@@\n@r2\nAC\n+\n@#\n"
    a = orc.encode(rec, kind=1)
    rc, out, offs = orc.read_lookup(a, [1, 0, 1])
    assert rc == 0 and out == b"@r2\nAC\n+\n@#\n@r1\nACGT\n+\n@@@@\n@r2\nAC\n+\n@#\n"
    assert list(offs) == [0, 12, 28, 40]
    with pytest.raises(RuntimeError):
        orc.encode(rec[:-3], kind=1)          # trailing partial record


def test_levels_and_deps_recomputed(orc, fq):
    """Stored deps/levels equal those recomputed from the decoded sequences."""
    x, _, a = fq
    p = orc.parse(x, **FASTQ_PARAMS)
    i = orc.info(a)
    off_dir = int.from_bytes(a[64:72], "little")
    off_dp = int.from_bytes(a[72:80], "little")
    off_di = int.from_bytes(a[80:88], "little")
    nb = i.n_blocks
    dp = np.frombuffer(a[off_dp:off_dp + 8 * (nb + 1)], dtype=np.uint64)
    di = np.frombuffer(a[off_di:off_di + 4 * int(dp[-1])], dtype=np.uint32)
    deps = {b: set() for b in range(nb)}
    pos = {b: b << 14 for b in range(nb)}
    for b, L, M, O in zip(p["blk"], p["ll"], p["ml"], p["of"]):
        b = int(b); pos[b] += int(L)
        if M and int(O) < (b << 14):
            hi = min(int(O) + int(M), b << 14)
            deps[b] |= set(range(int(O) >> 14, ((hi - 1) >> 14) + 1))
        pos[b] += int(M)
    lv = []
    for b in range(nb):
        assert sorted(deps[b]) == [int(v) for v in di[int(dp[b]):int(dp[b + 1])]]
        lv.append(0 if not deps[b] else 1 + max(lv[d] for d in deps[b]))
        stored = int.from_bytes(a[off_dir + 32 * b + 20:off_dir + 32 * b + 22], "little")
        assert stored == lv[b] < i.max_level
    assert i.n_levels == max(lv) + 1


def test_range_decode(orc, fq):
    x, _, a = fq
    rng = np.random.default_rng(4)
    B = 1 << 14
    N = len(x)
    cases = [(0, 0), (0, 1), (0, N), (N - 1, 1), (N, 0), (B - 1, 2), (B, B), (B - 1, B + 2),
             (3 * B, 1), (2 * B + 5, 3 * B)]
    cases += [(int(o), int(rng.integers(0, N - o + 1))) for o in rng.integers(0, N, 20)]
    scratch = np.empty(N, dtype=np.uint8)
    for o, L in cases:
        rc, out, cb = orc.decode_range(a, o, L, scratch)
        assert rc == 0 and out == x[o:o + L], (o, L)
    rc, _, _ = orc.decode_range(a, N, 1, scratch)
    assert rc == orc.ERANGE
    rc, _, _ = orc.decode_range(a, 5, N, scratch)
    assert rc == orc.ERANGE


def test_read_lookup_matches_records(orc, fq):
    x, starts, a = fq
    ids = np.array([0, 5, 5, 1499, 700, 3], dtype=np.int64)
    rc, out, offs = orc.read_lookup(a, ids)
    assert rc == 0
    exp = b"".join(x[int(starts[r]):int(starts[r + 1])] for r in ids)
    assert out == exp
    assert list(offs) == [0] + list(np.cumsum([int(starts[r + 1] - starts[r]) for r in ids]))
    rc, _, _ = orc.read_lookup(a, [1500])
    assert rc == orc.ERANGE
    rc, _, _ = orc.read_lookup(a, [-1])
    assert rc == orc.ERANGE
    plain = orc.encode(b"ACGT" * 100)
    rc, _, _ = orc.read_lookup(plain, [0])
    assert rc == orc.ENOINDEX


def _set64(a, off, v):
    b = bytearray(a)
    b[off:off + 8] = int(v).to_bytes(8, "little")
    return _rehash(b)


def _rehash(b):
    b[120:128] = brute.fnv1a64(bytes(b[:120])).to_bytes(8, "little")
    return bytes(b)


def test_validator_rejects_corruption(orc, fq):
    x, _, a = fq
    assert orc.validate(a) == 0
    bad = bytearray(a); bad[0] ^= 1
    assert orc.validate(bytes(bad)) == orc.EFORMAT                   # magic
    bad = bytearray(a); bad[30] ^= 1
    assert orc.validate(bytes(bad)) == orc.EFORMAT                   # header checksum
    assert orc.validate(a[:-1]) == orc.EFORMAT                       # truncated
    assert orc.validate(_set64(a, 24, len(x) + 1)) == orc.EFORMAT    # N vs n_blocks / width
    i = orc.info(a)
    off_dir = int.from_bytes(a[64:72], "little")
    off_dp = int.from_bytes(a[72:80], "little")
    off_di = int.from_bytes(a[80:88], "little")
    nb = i.n_blocks
    # wrong level in the directory
    b = next(k for k in range(nb) if int.from_bytes(a[off_dir + 32 * k + 20:off_dir + 32 * k + 22], "little") > 0)
    bad = bytearray(a)
    bad[off_dir + 32 * b + 20] ^= 1
    assert orc.validate(bytes(bad)) == orc.EFORMAT
    # a dependency on a later block
    dp = np.frombuffer(a[off_dp:off_dp + 8 * (nb + 1)], dtype=np.uint64)
    k = int(dp[b])
    bad = bytearray(a)
    bad[off_di + 4 * k:off_di + 4 * k + 4] = int(b).to_bytes(4, "little")
    assert orc.validate(bytes(bad)) == orc.EFORMAT
    # read index not increasing
    off_r = int.from_bytes(a[96:104], "little")
    bad = bytearray(a)
    bad[off_r + 8:off_r + 16] = (0).to_bytes(8, "little")
    assert orc.validate(bytes(bad)) == orc.EFORMAT


def test_payload_corruption_detected(orc, fq):
    x, _, a = fq
    off_pay = int.from_bytes(a[88:96], "little")
    off_r = int.from_bytes(a[96:104], "little")
    rng = np.random.default_rng(8)
    for pos in rng.integers(off_pay, off_r, 40):
        bad = bytearray(a)
        bad[int(pos)] ^= 0xFF
        rc, out = orc.decode(bytes(bad))
        assert rc in (orc.ECORRUPT, orc.EFORMAT) or out == x  # padding bytes are free
