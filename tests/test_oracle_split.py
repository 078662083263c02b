"""Pins of the stream-separated FASTQ oracle (oracle/split.py) against the
definition in the paper's Discussion ("Where ACEAPEX Stands on Ratio": ids,
sequences and qualities stored apart): hand-worked streams and tables
(tests/golden/split_fastq.json), record starts from a brute-force line scan,
round trips through the oracle codec, and the inputs the container refuses."""
import json
import os
import struct

import numpy as np
import pytest

import oracle
import oracle.split as sp
from gen.fastq import fastq

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "split_fastq.json")))
P = dict(block_log2=10, max_level=8, min_match=16, hash_len=16, hash_bits=16, chain_depth=16,
         window_log2=0, lit_lanes=64, seq_lanes=16, prob_bits=(11, 10, 10, 10), level_penalty=8)


def line_scan_starts(text: bytes) -> list:
    """Brute force: byte offset of every fourth line start, and len(text)."""
    starts, line = [], 0
    pos = 0
    while pos < len(text):
        if line % 4 == 0:
            starts.append(pos)
        nl = text.index(b"\n", pos)
        pos = nl + 1
        line += 1
    return starts + [len(text)]


@pytest.mark.parametrize("case", range(len(GOLDEN["cases"])))
def test_hand_worked_streams(case):
    c = GOLDEN["cases"][case]
    st = sp.fastq_streams(c["text"].encode())
    for k in sp.STREAMS:
        assert st[k] == c[k].encode(), k
    assert st["hstart"].tolist() == c["hstart"]
    assert st["sstart"].tolist() == c["sstart"]
    assert sp.record_starts(st["hstart"], st["sstart"]).tolist() == c["record_starts"]
    assert sp.join(st) == c["text"].encode()


@pytest.mark.parametrize("text", GOLDEN["rejected"])
def test_refused_inputs(text):
    with pytest.raises(ValueError):
        sp.fastq_streams(text.encode())


def test_record_starts_match_line_scan():
    x, starts = fastq(n_records=300, seed=11)
    x = bytes(x)
    st = sp.fastq_streams(x)
    R = sp.record_starts(st["hstart"], st["sstart"])
    assert R.tolist() == line_scan_starts(x)
    assert R.tolist() == [int(v) for v in starts]          # the generator's own record starts
    assert sp.join(st) == x
    # each stream is every fourth line
    lines = x.split(b"\n")[:-1]
    for k, name in enumerate(sp.STREAMS):
        assert st[name] == b"".join(l + b"\n" for l in lines[k::4])


def test_container_round_trip_and_header():
    x, _ = fastq(n_records=400, seed=12)
    x = bytes(x)
    buf = sp.encode(x, **P)
    assert buf[:4] == b"LZSF"
    version, flags, n, n_reads = struct.unpack_from("<HHQQ", buf, 4)
    assert (version, flags, n, n_reads) == (2, 3, len(x), 400)
    assert struct.unpack_from("<Q", buf, 120)[0] == oracle.fnv1a64(buf[:120])
    assert struct.unpack_from("<Q", buf, 104)[0] == oracle.fnv1a64(x)
    c = sp.parse(buf)
    assert all(o % 256 == 0 for o in c["sub_off"])
    st = sp.fastq_streams(x)
    for k, a in zip(sp.STREAMS, c["subs"]):
        rc, data = oracle.decode(a)
        assert rc == 0 and data == st[k], k
        assert oracle.info(a).kind == 0
    R = sp.record_starts(c["hstart"], c["sstart"])
    assert c["max_record_len"] == int(np.max(np.diff(R)))
    assert sp.decode(buf) == x
    assert sp.decode_range(buf, 1000, 5000) == x[1000:6000]
    ids = [0, 399, 17, 17, 250]
    assert sp.read_lookup(buf, ids) == [x[int(R[i]):int(R[i + 1])] for i in ids]


def test_empty_container():
    buf = sp.encode(b"", **P)
    assert sp.decode(buf) == b""
    assert sp.parse(buf)["n_reads"] == 0


def test_bad_header_refused():
    x, _ = fastq(n_records=20, seed=13)
    buf = bytearray(sp.encode(bytes(x), **P))
    buf[8] ^= 1                                            # N changed, header hash stale
    with pytest.raises(ValueError):
        sp.parse(bytes(buf))
