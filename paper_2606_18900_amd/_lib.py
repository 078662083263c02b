"""ctypes binding of liblz.so (the C ABI in include/lz.h): argument marshalling
only.  Raises ImportError-like RuntimeError when the library is not built —
there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LZ_STAGE_CLOCKS=1 loads the instrumented build (liblz_clk.so, built by
# `python -m paper_2606_18900_amd.build --stage-clocks`) for stage profiling.
LIB_PATH = os.path.join(HERE, "liblz_clk.so" if os.environ.get("LZ_STAGE_CLOCKS") == "1" else "liblz.so")

LZ_OK, LZ_EINVAL, LZ_EFORMAT, LZ_ECAPACITY, LZ_ERANGE = 0, -1, -2, -3, -4
LZ_ENOINDEX, LZ_EDEVICE, LZ_ECORRUPT, LZ_EBUDGET = -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES, NOALLOC_MAX_IDS = 32 << 20, 4096   # lz.h LZ_NOALLOC_*
NAMES = {0: "LZ_OK", -1: "LZ_EINVAL", -2: "LZ_EFORMAT", -3: "LZ_ECAPACITY", -4: "LZ_ERANGE",
         -5: "LZ_ENOINDEX", -6: "LZ_EDEVICE", -7: "LZ_ECORRUPT", -8: "LZ_EBUDGET"}

# every symbol include/lz.h declares
EXPORTS = ["lz_params_default", "lz_encode", "lz_free", "lz_info_get", "lz_open", "lz_close",
           "lz_get_info", "lz_set_tuning", "lz_get_tuning", "lz_decode_all", "lz_decode_range",
           "lz_read_lookup", "lz_read_lookup_noalloc", "lz_fasta_index", "lz_decode_region", "lz_decode_batch", "lz_verify", "lz_verify_range", "lz_last_stats", "lz_sync_status", "lz_last_error",
           "lz_encode_split", "lz_split_info_get", "lz_split_open", "lz_split_close", "lz_split_stream",
           "lz_split_decode_all", "lz_split_scratch_bytes", "lz_split_decode_range",
           "lz_split_read_lookup", "lz_split_sync_status"]


class LzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (NAMES.get(code, str(code)), msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("block_log2", C.c_uint32), ("max_level", C.c_uint32),
                ("min_match", C.c_uint32), ("hash_len", C.c_uint32),
                ("hash_bits", C.c_uint32), ("chain_depth", C.c_uint32),
                ("window_log2", C.c_uint32), ("lit_lanes", C.c_uint32),
                ("seq_lanes", C.c_uint32), ("prob_bits", C.c_uint32 * 4),
                ("kind", C.c_uint32), ("level_penalty", C.c_uint32),
                ("threads", C.c_uint32), ("segment_log2", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_uint64), ("n_blocks", C.c_uint64), ("n_reads", C.c_uint64),
                ("archive_len", C.c_uint64), ("source_fnv", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("literal_bytes", C.c_uint64),
                ("payload_bytes", C.c_uint64), ("block_log2", C.c_uint32),
                ("max_level", C.c_uint32), ("n_levels", C.c_uint32),
                ("offset_width", C.c_uint32), ("max_record_len", C.c_uint32),
                ("kind", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int64), ("a", C.c_int64), ("b", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("closure_blocks", C.c_uint64), ("scratch_slots", C.c_uint64), ("covering", C.c_uint64)]


class FastaSeq(C.Structure):
    _fields_ = [("name", C.c_char * 64), ("offset", C.c_uint64), ("length", C.c_uint64),
                ("line_bases", C.c_uint32), ("line_bytes", C.c_uint32)]


class SplitInfo(C.Structure):
    _fields_ = [("n", C.c_uint64), ("n_reads", C.c_uint64), ("container_len", C.c_uint64),
                ("source_fnv", C.c_uint64), ("workspace_bytes", C.c_uint64),
                ("stream_len", C.c_uint64 * 4), ("archive_len", C.c_uint64 * 4),
                ("max_record_len", C.c_uint32), ("reserved", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("sync_mode", C.c_uint32), ("wg_per_cu", C.c_uint32), ("spin_limit", C.c_uint32),
                ("req_sync_mode", C.c_uint32), ("plan_blocks", C.c_uint32)]


_lib = None


def lib():
    """Load liblz.so (built by __graft_entry__.build / paper_2606_18900_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblz.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        L.lz_last_error.restype = C.c_char_p
        L.lz_encode.argtypes = [vp, u64, vp, vp, vp]
        L.lz_info_get.argtypes = [vp, u64, vp]
        L.lz_open.argtypes = [vp, u64, vp, u64, vp, vp]
        L.lz_close.argtypes = [vp]
        L.lz_get_info.argtypes = [vp, vp]
        L.lz_set_tuning.argtypes = [vp, vp]
        L.lz_get_tuning.argtypes = [vp, vp]
        L.lz_decode_all.argtypes = [vp, vp, u64, vp]
        L.lz_decode_range.argtypes = [vp, u64, u64, vp, vp, u64, vp]
        L.lz_read_lookup.argtypes = [vp, vp, u64, vp, u64, vp, vp, u64, vp]
        L.lz_read_lookup_noalloc.argtypes = [vp, vp, u64, vp, u64, vp, vp]
        L.lz_fasta_index.argtypes = [vp, u64, vp, u64, vp]
        L.lz_decode_region.argtypes = [vp, vp, u64, u64, vp, vp, u64, vp]
        L.lz_decode_batch.argtypes = [vp, vp, vp, u64, vp, u64, vp, vp, u64, vp]
        L.lz_verify.argtypes = [vp, vp, vp, vp, u64, vp]
        L.lz_verify_range.argtypes = [vp, vp, u64, u64, vp, u64, vp]
        L.lz_last_stats.argtypes = [vp, vp, vp]
        L.lz_sync_status.argtypes = [vp, vp]
        L.lz_free.argtypes = [vp]
        L.lz_params_default.argtypes = [vp]
        L.lz_encode_split.argtypes = [vp, u64, vp, vp, vp]
        L.lz_split_info_get.argtypes = [vp, u64, vp, vp]
        L.lz_split_open.argtypes = [vp, u64, vp, u64, vp, vp]
        L.lz_split_close.argtypes = [vp]
        L.lz_split_stream.argtypes = [vp, u32, vp]
        L.lz_split_decode_all.argtypes = [vp, vp, u64, vp]
        L.lz_split_scratch_bytes.argtypes = [vp, u64, vp]
        L.lz_split_decode_range.argtypes = [vp, u64, u64, vp, vp, u64, vp]
        L.lz_split_read_lookup.argtypes = [vp, vp, u64, vp, u64, vp, vp, u64, vp]
        L.lz_split_sync_status.argtypes = [vp, vp]
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != LZ_OK:
        raise LzError(rc, lib().lz_last_error().decode(errors="replace"))


def default_params(**kw) -> Params:
    p = Params()
    check(lib().lz_params_default(C.byref(p)))
    for k, v in kw.items():
        if k == "prob_bits":
            for i, b in enumerate(v):
                p.prob_bits[i] = b
        else:
            setattr(p, k, v)
    return p
