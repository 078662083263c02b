"""Stream-separated FASTQ container, plain definition (CPU, slow, obvious).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

The paper (Discussion, "Where ACEAPEX Stands on Ratio") reports that storing
read ids, sequences and quality strings apart, as separate archives of the
same codec, gains ratio because each group is homogeneous.  This module is
that statement written out for 4-line FASTQ records:

  stream H: every record's first line (the '@' id line) with its newline
  stream S: every record's second line (bases) with its newline
  stream P: every record's third line ('+') with its newline
  stream Q: every record's fourth line (qualities) with its newline

Each stream is one ordinary archive (kind 0).  Reassembly goes through a read
index: for record i, hstart[i] and sstart[i] are the offsets of its lines in
streams H and S (n_reads + 1 entries each, the last one the stream length).
This container only takes files whose third lines are exactly "+" and whose
quality lines are as long as their sequence lines, so that record i's P and
Q lines start at 2 i and sstart[i]; its first byte in the original file is
hstart[i] + 2 sstart[i] + 2 i.

Container layout (all integers little-endian):
   0  "LZSF"            4  u16 version = 2      6  u16 flags = 3
   8  u64 N            16  u64 n_reads
  24  u64 offset of hstart[]       32  u64 offset of sstart[]
  40  u64 sub-archive offsets [4] (H, S, P, Q; multiples of 256)
  72  u64 sub-archive lengths [4]
 104  u64 FNV-1a-64 of the source  112  u32 longest record  116  u32 0
 120  u64 FNV-1a-64 of bytes 0..119
 128  hstart[], sstart[] (u64), then each sub-archive at its offset; gaps
      are zero bytes.
"""
from __future__ import annotations

import struct

import numpy as np

from . import decode as _decode
from . import encode as _encode
from . import fnv1a64

MAGIC = b"LZSF"
VERSION = 2
FLAGS = 3
HEADER = 128
STREAMS = ("H", "S", "P", "Q")


def fastq_streams(text: bytes) -> dict:
    """Split a FASTQ text into its four line streams and the two record
    tables.  ValueError if the text is not whole 4-line records ending in
    newlines, an id line lacks '@', a third line is not exactly '+', or a
    quality line's length differs from its sequence line's."""
    text = bytes(text)
    if text and not text.endswith(b"\n"):
        raise ValueError("FASTQ text must end with a newline")
    lines = text.split(b"\n")[:-1] if text else []
    if len(lines) % 4:
        raise ValueError("FASTQ text must hold whole 4-line records")
    parts = {k: [] for k in STREAMS}
    hstart, sstart = [0], [0]
    for r in range(len(lines) // 4):
        l1, l2, l3, l4 = lines[4 * r: 4 * r + 4]
        if not l1.startswith(b"@"):
            raise ValueError("record %d: id line does not start with '@'" % r)
        if l3 != b"+":
            raise ValueError("record %d: third line is not a bare '+'" % r)
        if len(l4) != len(l2):
            raise ValueError("record %d: quality and sequence lengths differ" % r)
        for k, line in zip(STREAMS, (l1, l2, l3, l4)):
            parts[k].append(line + b"\n")
        hstart.append(hstart[-1] + len(l1) + 1)
        sstart.append(sstart[-1] + len(l2) + 1)
    out = {k: b"".join(v) for k, v in parts.items()}
    out["hstart"] = np.array(hstart, dtype=np.uint64)
    out["sstart"] = np.array(sstart, dtype=np.uint64)
    return out


def record_starts(hstart, sstart) -> np.ndarray:
    """First byte of every record in the original file (and its length at the
    end): hstart[i] + 2 sstart[i] + 2 i."""
    i = np.arange(len(hstart), dtype=np.uint64)
    return np.asarray(hstart, dtype=np.uint64) + 2 * np.asarray(sstart, dtype=np.uint64) + 2 * i


def join(st: dict) -> bytes:
    """Reassemble the FASTQ text from the four streams and the record tables."""
    h, s = st["hstart"], st["sstart"]
    out = []
    for i in range(len(h) - 1):
        out.append(st["H"][int(h[i]):int(h[i + 1])])
        out.append(st["S"][int(s[i]):int(s[i + 1])])
        out.append(st["P"][2 * i: 2 * i + 2])
        out.append(st["Q"][int(s[i]):int(s[i + 1])])
    return b"".join(out)


def _pad(n: int, a: int = 256) -> int:
    return (n + a - 1) // a * a


def encode(text: bytes, **params) -> bytes:
    """The container of `text`; every stream is encoded by the oracle encoder
    with `params` and kind 0 (no read index of its own)."""
    text = bytes(text)
    st = fastq_streams(text)
    p = dict(params)
    p["kind"] = 0
    subs = [_encode(st[k], **p) for k in STREAMS]
    n_reads = len(st["hstart"]) - 1
    R = record_starts(st["hstart"], st["sstart"])
    longest = int(np.max(np.diff(R))) if n_reads else 0
    off_h = HEADER
    off_s = off_h + 8 * (n_reads + 1)
    o = _pad(off_s + 8 * (n_reads + 1))
    sub_off = []
    for a in subs:
        sub_off.append(o)
        o = _pad(o + len(a))
    total = sub_off[-1] + len(subs[-1])
    buf = bytearray(total)
    head = MAGIC + struct.pack("<HHQQQQ", VERSION, FLAGS, len(text), n_reads, off_h, off_s)
    head += struct.pack("<4Q", *sub_off) + struct.pack("<4Q", *[len(a) for a in subs])
    head += struct.pack("<QII", fnv1a64(text), longest, 0)
    assert len(head) == 120
    buf[:120] = head
    buf[120:128] = struct.pack("<Q", fnv1a64(head))
    buf[off_h:off_s] = st["hstart"].astype("<u8").tobytes()
    buf[off_s:off_s + 8 * (n_reads + 1)] = st["sstart"].astype("<u8").tobytes()
    for a, so in zip(subs, sub_off):
        buf[so:so + len(a)] = a
    return bytes(buf)


def parse(buf: bytes) -> dict:
    """Header fields, record tables and sub-archive byte strings of a
    container.  ValueError on a bad magic, version, flags or header hash."""
    buf = bytes(buf)
    if len(buf) < HEADER or buf[:4] != MAGIC:
        raise ValueError("not a split FASTQ container")
    version, flags, n, n_reads, off_h, off_s = struct.unpack_from("<HHQQQQ", buf, 4)
    if version != VERSION or flags != FLAGS:
        raise ValueError("unsupported version or flags")
    if struct.unpack_from("<Q", buf, 120)[0] != fnv1a64(buf[:120]):
        raise ValueError("header hash mismatch")
    sub_off = struct.unpack_from("<4Q", buf, 40)
    sub_len = struct.unpack_from("<4Q", buf, 72)
    src_fnv, longest, _ = struct.unpack_from("<QII", buf, 104)
    hs = np.frombuffer(buf, dtype="<u8", count=n_reads + 1, offset=off_h).astype(np.uint64)
    ss = np.frombuffer(buf, dtype="<u8", count=n_reads + 1, offset=off_s).astype(np.uint64)
    return {"n": n, "n_reads": n_reads, "hstart": hs, "sstart": ss, "source_fnv": src_fnv,
            "max_record_len": longest,
            "subs": [buf[o:o + ln] for o, ln in zip(sub_off, sub_len)],
            "sub_off": sub_off, "sub_len": sub_len}


def decode(buf: bytes) -> bytes:
    """Whole-file decode: every stream by the oracle decoder, then join."""
    c = parse(buf)
    st = {"hstart": c["hstart"], "sstart": c["sstart"]}
    for k, a in zip(STREAMS, c["subs"]):
        rc, data = _decode(a)
        if rc:
            raise ValueError("stream %s: oracle decode failed (%d)" % (k, rc))
        st[k] = data
    return join(st)


def decode_range(buf: bytes, offset: int, length: int) -> bytes:
    """Bytes [offset, offset + length) of the original file."""
    return decode(buf)[offset: offset + length]


def read_lookup(buf: bytes, ids) -> list:
    """Records `ids` of the original file (each with its four lines)."""
    c = parse(buf)
    x = decode(buf)
    R = record_starts(c["hstart"], c["sstart"])
    return [x[int(R[i]):int(R[i + 1])] for i in ids]
