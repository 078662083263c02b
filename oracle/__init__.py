"""ctypes access to the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

OK, EINVAL, EFORMAT, ECAPACITY, ERANGE, ENOINDEX, ECORRUPT = 0, -1, -2, -3, -4, -5, -7


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP for the level-parallel timer)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("block_log2", C.c_uint32), ("max_level", C.c_uint32),
                ("min_match", C.c_uint32), ("hash_len", C.c_uint32),
                ("hash_bits", C.c_uint32), ("chain_depth", C.c_uint32),
                ("window_log2", C.c_uint32), ("lit_lanes", C.c_uint32),
                ("seq_lanes", C.c_uint32), ("prob_bits", C.c_uint32 * 4),
                ("kind", C.c_uint32), ("level_penalty", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_uint64), ("n_blocks", C.c_uint64), ("n_reads", C.c_uint64),
                ("total_len", C.c_uint64), ("source_fnv", C.c_uint64),
                ("block_log2", C.c_uint32), ("max_level", C.c_uint32),
                ("n_levels", C.c_uint32), ("offset_width", C.c_uint32),
                ("max_record_len", C.c_uint32), ("kind", C.c_uint32)]


_lib = None
u8p = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        L.orc_fnv1a64.restype = C.c_uint64
        L.orc_fnv1a64.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64]
        L.orc_fnv_basis.restype = C.c_uint64
        _lib = L
    return _lib


def params(**kw) -> Params:
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "prob_bits":
            for i, b in enumerate(v):
                p.prob_bits[i] = b
        else:
            setattr(p, k, v)
    return p


def _buf(data):
    if isinstance(data, np.ndarray):
        a = np.ascontiguousarray(data, dtype=np.uint8)
    else:
        a = np.frombuffer(bytes(data), dtype=np.uint8)
    return a, (a.ctypes.data if a.size else 0)


def fnv1a64(data, h: int | None = None) -> int:
    a, p = _buf(data)
    return int(lib().orc_fnv1a64(C.c_void_p(p), a.size,
                                 lib().orc_fnv_basis() if h is None else h))


def encode(data, **kw) -> bytes:
    a, p = _buf(data)
    out = C.POINTER(C.c_uint8)()
    n = C.c_uint64()
    rc = lib().orc_encode(C.c_void_p(p), C.c_uint64(a.size), C.byref(params(**kw)),
                          C.byref(out), C.byref(n))
    if rc:
        raise RuntimeError("orc_encode rc=%d" % rc)
    res = C.string_at(out, n.value)
    lib().orc_free(out)
    return res


def parse(data, **kw):
    """Greedy parse: dict of numpy arrays blk, ll, ml, of and per-block level."""
    a, p = _buf(data)
    ns = C.c_uint64()
    blk, ll, ml = C.POINTER(C.c_uint32)(), C.POINTER(C.c_uint32)(), C.POINTER(C.c_uint32)()
    of, lv = C.POINTER(C.c_uint64)(), C.POINTER(C.c_uint16)()
    pr = params(**kw)
    rc = lib().orc_parse(C.c_void_p(p), C.c_uint64(a.size), C.byref(pr), C.byref(ns),
                         C.byref(blk), C.byref(ll), C.byref(ml), C.byref(of), C.byref(lv))
    if rc:
        raise RuntimeError("orc_parse rc=%d" % rc)
    n = ns.value
    B = 1 << pr.block_log2
    nb = (a.size + B - 1) // B
    res = {
        "blk": np.ctypeslib.as_array(blk, (n,)).copy() if n else np.zeros(0, np.uint32),
        "ll": np.ctypeslib.as_array(ll, (n,)).copy() if n else np.zeros(0, np.uint32),
        "ml": np.ctypeslib.as_array(ml, (n,)).copy() if n else np.zeros(0, np.uint32),
        "of": np.ctypeslib.as_array(of, (n,)).copy() if n else np.zeros(0, np.uint64),
        "level": np.ctypeslib.as_array(lv, (nb,)).copy() if nb else np.zeros(0, np.uint16),
    }
    for q in (blk, ll, ml, of, lv):
        lib().orc_free(q)
    return res


def rebase(parsed: dict, block_log2: int) -> np.ndarray:
    """Sources after the encoder's rebasing step (orc_rebase) applied to a
    parse as returned by parse(); returns the new offsets."""
    of = np.ascontiguousarray(parsed["of"], dtype=np.uint64).copy()
    blk = np.ascontiguousarray(parsed["blk"], dtype=np.uint32)
    ll = np.ascontiguousarray(parsed["ll"], dtype=np.uint32)
    ml = np.ascontiguousarray(parsed["ml"], dtype=np.uint32)
    n = len(of)
    if n:
        lib().orc_rebase(C.c_uint64(n), C.c_void_p(blk.ctypes.data), C.c_void_p(ll.ctypes.data),
                         C.c_void_p(ml.ctypes.data), C.c_void_p(of.ctypes.data), C.c_uint32(block_log2))
    return of


def info(archive: bytes) -> Info:
    a, p = _buf(archive)
    i = Info()
    rc = lib().orc_info_get(C.c_void_p(p), C.c_uint64(a.size), C.byref(i))
    if rc:
        raise RuntimeError("orc_info rc=%d" % rc)
    return i


def validate(archive) -> int:
    a, p = _buf(archive)
    return int(lib().orc_validate(C.c_void_p(p), C.c_uint64(a.size)))


def decode(archive, out: np.ndarray | None = None) -> tuple[int, bytes | None]:
    a, p = _buf(archive)
    rc0 = validate(a)
    if rc0:
        return rc0, None
    n = info(a).n
    o = np.empty(max(n, 1), dtype=np.uint8) if out is None else out
    rc = lib().orc_decode(C.c_void_p(p), C.c_uint64(a.size), C.c_void_p(o.ctypes.data),
                          C.c_uint64(n))
    return rc, (o[:n].tobytes() if rc == 0 and out is None else None)


def decode_levels(archive, out: np.ndarray, threads: int) -> int:
    a, p = _buf(archive)
    return int(lib().orc_decode_levels(C.c_void_p(p), C.c_uint64(a.size),
                                       C.c_void_p(out.ctypes.data), C.c_uint64(out.size),
                                       C.c_int(threads)))


def decode_range(archive, off: int, length: int, scratch: np.ndarray | None = None):
    a, p = _buf(archive)
    n = info(a).n
    s = np.empty(max(n, 1), dtype=np.uint8) if scratch is None else scratch
    o = np.empty(max(length, 1), dtype=np.uint8)
    cb = C.c_uint64()
    rc = lib().orc_decode_range(C.c_void_p(p), C.c_uint64(a.size), C.c_uint64(off),
                                C.c_uint64(length), C.c_void_p(s.ctypes.data),
                                C.c_void_p(o.ctypes.data), C.byref(cb))
    return rc, (o[:length].tobytes() if rc == 0 else None), cb.value


def read_lookup(archive, ids, scratch: np.ndarray | None = None):
    a, p = _buf(archive)
    inf = info(a)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    s = np.empty(max(inf.n, 1), dtype=np.uint8) if scratch is None else scratch
    cap = max(1, ids.size * max(1, inf.max_record_len))
    o = np.empty(cap, dtype=np.uint8)
    offs = np.zeros(ids.size + 1, dtype=np.uint64)
    rc = lib().orc_read_lookup(C.c_void_p(p), C.c_uint64(a.size),
                               C.c_void_p(ids.ctypes.data if ids.size else 0),
                               C.c_uint64(ids.size), C.c_void_p(s.ctypes.data),
                               C.c_void_p(o.ctypes.data), C.c_uint64(cap),
                               C.c_void_p(offs.ctypes.data))
    if rc:
        return rc, None, None
    return rc, o[: int(offs[-1])].tobytes(), offs


def normalize(counts, prob_bits: int):
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    f = np.zeros(256, dtype=np.uint16)
    rc = lib().orc_normalize(C.c_void_p(c.ctypes.data), C.c_uint32(prob_bits),
                             C.c_void_p(f.ctypes.data))
    return rc, f


def rans_lanes(n: int, max_lanes: int, per_lane: int = 16) -> int:
    return int(lib().orc_rans_lanes(C.c_uint32(n), C.c_uint32(max_lanes), C.c_uint32(per_lane)))


def rans_encode(sym, freq, prob_bits: int, lanes: int):
    a, p = _buf(sym)
    f = np.ascontiguousarray(freq, dtype=np.uint16)
    body = C.POINTER(C.c_uint8)()
    bl, nw = C.c_uint64(), C.c_uint32()
    rc = lib().orc_rans_encode(C.c_void_p(p), C.c_uint32(a.size), C.c_void_p(f.ctypes.data),
                               C.c_uint32(prob_bits), C.c_uint32(lanes), C.byref(body),
                               C.byref(bl), C.byref(nw))
    if rc:
        return rc, None, 0
    res = C.string_at(body, bl.value)
    lib().orc_free(body)
    return rc, res, nw.value


def rans_decode(body: bytes, n: int, n_words: int, freq, prob_bits: int, lanes: int):
    a, p = _buf(body)
    f = np.ascontiguousarray(freq, dtype=np.uint16)
    o = np.empty(max(n, 1), dtype=np.uint8)
    rc = lib().orc_rans_decode(C.c_void_p(p), C.c_uint64(a.size), C.c_uint32(n),
                               C.c_uint32(n_words), C.c_void_p(f.ctypes.data),
                               C.c_uint32(prob_bits), C.c_uint32(lanes),
                               C.c_void_p(o.ctypes.data))
    return rc, (o[:n].tobytes() if rc == 0 else None)


def fasta_sequences(text: bytes) -> dict:
    """Plain definition of a FASTA file's sequences: a record is a '>' line
    whose name is the text up to the first space or tab, followed by lines
    whose concatenation (newlines removed) is the sequence.  Returns
    {name: (sequence bytes, byte offset of its first base)}."""
    out = {}
    pos = 0
    for rec in text.split(b"\n>"):
        start = pos
        pos += len(rec) + 2                    # the "\n>" separator
        if start == 0:
            assert rec.startswith(b">")
            rec = rec[1:]
            start = 1
        head, _, body = rec.partition(b"\n")
        name = head.split(b" ")[0].split(b"\t")[0].decode()
        out[name] = (body.replace(b"\n", b""), start + len(head) + 1)
    return out


def fasta_region(text: bytes, name: str, start: int, end: int) -> bytes:
    """Bases [start, end) of sequence `name` (plain definition: slice of the
    concatenated sequence lines); the coordinate access the paper names as
    future work in its Read-Level Index subsection."""
    return fasta_sequences(text)[name][0][start:end]
