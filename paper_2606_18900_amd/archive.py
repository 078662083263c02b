"""Python face of liblz: host encode, and an Archive bound on the GPU whose
decode calls enqueue HIP kernels on the current torch stream.  torch provides
device memory and streams only; every decode step runs in liblz's kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


def encode(data, **params) -> bytes:
    """Compress host bytes (lz_encode).  Keyword arguments override the
    default lz_params fields (kind, min_match, level_penalty, ...)."""
    if isinstance(data, np.ndarray):
        a = np.ascontiguousarray(data, dtype=np.uint8)
    else:
        a = np.frombuffer(memoryview(data), dtype=np.uint8)
    p = _lib.default_params(**params)
    out = C.c_void_p()
    n = C.c_uint64()
    check(lib().lz_encode(C.c_void_p(a.ctypes.data if a.size else 0), a.size, C.byref(p),
                          C.byref(out), C.byref(n)))
    try:
        if not n.value:
            return b""
        return bytes(memoryview((C.c_char * n.value).from_address(out.value)))   # any size
    finally:
        lib().lz_free(out)


def fasta_index(data) -> list:
    """lz_fasta_index: .fai-style description (name, offset, length, line
    widths) of every sequence of a FASTA text, for lz_decode_region."""
    a = np.frombuffer(memoryview(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    cnt = C.c_uint64()
    check(lib().lz_fasta_index(C.c_void_p(a.ctypes.data if a.size else 0), a.size, None, 0, C.byref(cnt)))
    arr = (_lib.FastaSeq * max(1, cnt.value))()
    check(lib().lz_fasta_index(C.c_void_p(a.ctypes.data if a.size else 0), a.size, arr, cnt.value,
                               C.byref(cnt)))
    return list(arr[: cnt.value])


def info(archive: bytes) -> _lib.Info:
    i = _lib.Info()
    a = np.frombuffer(memoryview(archive), dtype=np.uint8)
    check(lib().lz_info_get(C.c_void_p(a.ctypes.data), a.size, C.byref(i)))
    return i


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Archive:
    """An archive resident in HBM plus its decoder workspace (lz_open)."""

    def __init__(self, archive, device: str | torch.device = "cuda:0", stream=None):
        self.device = torch.device(device)
        if isinstance(archive, torch.Tensor):
            assert archive.dtype == torch.uint8 and archive.is_cuda and archive.is_contiguous()
            self.d_archive = archive
            head = archive[:128].cpu().numpy().tobytes()
        else:
            import warnings
            with warnings.catch_warnings():   # read-only host bytes: copied, never written
                warnings.simplefilter("ignore")
                host = torch.from_numpy(np.frombuffer(archive, dtype=np.uint8))
            self.d_archive = torch.empty(host.numel(), dtype=torch.uint8, device=self.device)
            self.d_archive.copy_(host)
            head = bytes(archive[:128])
        i = _lib.Info()
        check(lib().lz_info_get(head, len(head) if len(head) < 128 else self.d_archive.numel(), C.byref(i)))
        self.info = i
        self.ws = torch.empty(max(i.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        self.h = C.c_void_p()
        check(lib().lz_open(_ptr(self.d_archive), self.d_archive.numel(), _ptr(self.ws),
                            self.ws.numel(), _stream(stream), C.byref(self.h)))
        full = _lib.Info()
        check(lib().lz_get_info(self.h, C.byref(full)))
        self.literal_bytes = int(full.literal_bytes)
        self.payload_bytes = int(full.payload_bytes)

    # -- properties
    @property
    def n(self) -> int:
        return int(self.info.n)

    @property
    def n_blocks(self) -> int:
        return int(self.info.n_blocks)

    @property
    def n_reads(self) -> int:
        return int(self.info.n_reads)

    def close(self):
        if self.h:
            lib().lz_close(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning
    def tuning(self) -> _lib.Tuning:
        t = _lib.Tuning()
        check(lib().lz_get_tuning(self.h, C.byref(t)))
        return t

    def set_tuning(self, sync_mode: int | None = None, wg_per_cu: int | None = None,
                   spin_limit: int | None = None, req_sync_mode: int | None = None,
                   plan_blocks: int | None = None):
        t = self.tuning()
        for f, v in (("sync_mode", sync_mode), ("wg_per_cu", wg_per_cu), ("spin_limit", spin_limit),
                     ("req_sync_mode", req_sync_mode), ("plan_blocks", plan_blocks)):
            if v is not None:
                setattr(t, f, v)
        check(lib().lz_set_tuning(self.h, C.byref(t)))

    # -- decode
    def decode_all(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(self.n, 1), dtype=torch.uint8, device=self.device)
        check(lib().lz_decode_all(self.h, _ptr(out), out.numel(), _stream(stream)))
        return out[: self.n]

    def scratch_bytes(self, n_requests: int, n_slots: int | None = None) -> int:
        """Scratch for a request call: per-request spans and prefix sums, then
        n_slots block-sized slots (default: one per block, a bound on any
        closure)."""
        n = max(1, n_requests)
        head = (16 * n + 16 * (n + 1) + 255) & ~255
        slots = self.n_blocks if n_slots is None else n_slots
        return head + slots * (1 << int(self.info.block_log2))

    def _scratch(self, n_requests: int, scratch, n_slots=None) -> torch.Tensor:
        if scratch is None:
            scratch = torch.empty(self.scratch_bytes(n_requests, n_slots), dtype=torch.uint8,
                                  device=self.device)
        return scratch

    def decode_range(self, offset: int, length: int, out: torch.Tensor | None = None,
                     scratch: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(length, 1), dtype=torch.uint8, device=self.device)
        scratch = self._scratch(1, scratch)
        check(lib().lz_decode_range(self.h, offset, length, _ptr(out), _ptr(scratch),
                                    scratch.numel(), _stream(stream)))
        return out[:length]

    def read_lookup(self, ids, out: torch.Tensor | None = None,
                    offsets: torch.Tensor | None = None, scratch: torch.Tensor | None = None,
                    stream=None):
        ids = torch.as_tensor(ids, dtype=torch.int64, device=self.device).contiguous()
        n = ids.numel()
        cap = max(1, n * int(self.info.max_record_len))
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=self.device)
        if offsets is None:
            offsets = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        scratch = self._scratch(n, scratch)
        check(lib().lz_read_lookup(self.h, _ptr(ids), n, _ptr(out), out.numel(), _ptr(offsets),
                                   _ptr(scratch), scratch.numel(), _stream(stream)))
        return out, offsets

    def read_lookup_noalloc(self, ids: torch.Tensor, out: torch.Tensor, offsets: torch.Tensor,
                            stream=None):
        """lz_read_lookup_noalloc: read lookup whose request scratch is the
        library's fixed device array (no allocation by the call; ids, out and
        offsets are the caller's device tensors)."""
        assert ids.dtype == torch.int64 and ids.is_contiguous()
        check(lib().lz_read_lookup_noalloc(self.h, _ptr(ids), ids.numel(), _ptr(out), out.numel(),
                                           _ptr(offsets), _stream(stream)))
        return out, offsets

    def decode_region(self, seq: _lib.FastaSeq, start: int, end: int, out: torch.Tensor | None = None,
                      scratch: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """lz_decode_region: bases [start, end) of FASTA sequence `seq` (an
        entry of fasta_index), newlines removed."""
        n = end - start
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        if scratch is None:
            W = max(1, int(seq.line_bases))
            span = n + n // W + 2
            scratch = torch.empty(((span + 255) & ~255) + self.scratch_bytes(1, 4096), dtype=torch.uint8,
                                  device=self.device)
        check(lib().lz_decode_region(self.h, C.byref(seq), start, end, _ptr(out), _ptr(scratch),
                                     scratch.numel(), _stream(stream)))
        return out[:n]

    def decode_batch(self, reqs: torch.Tensor, n: torch.Tensor, n_max: int, out: torch.Tensor,
                     offsets: torch.Tensor, scratch: torch.Tensor, stream=None):
        """reqs: device int64 [n_max, 3] rows (kind, a, b); n: device int32 [1]
        holding the live request count (<= n_max)."""
        check(lib().lz_decode_batch(self.h, _ptr(reqs), _ptr(n), n_max, _ptr(out), out.numel(),
                                    _ptr(offsets), _ptr(scratch), scratch.numel(), _stream(stream)))

    def stream_range(self, offset: int, length: int, window: int,
                     out: torch.Tensor | None = None, scratch: torch.Tensor | None = None,
                     stream=None):
        """Range decode through a capped output window (Scale section: output
        larger than device memory).  Yields (window_offset, view) for consecutive
        windows of at most `window` bytes decoded into the same buffer; each
        view is valid until the next one is produced (the caller synchronises or
        consumes on the same stream).  Blocks an earlier window already dropped
        are decoded again into scratch when a later block needs them."""
        if out is None:
            out = torch.empty(window, dtype=torch.uint8, device=self.device)
        assert out.numel() >= window
        if scratch is None:
            scratch = self._scratch(1, scratch, n_slots=min(self.n_blocks, 65536))
        o = offset
        end = offset + length
        while o < end:
            w = min(window, end - o)
            check(lib().lz_decode_range(self.h, o, w, _ptr(out), _ptr(scratch), scratch.numel(),
                                        _stream(stream)))
            yield o, out[:w]
            o += w

    def verify(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        tree = torch.zeros(1, dtype=torch.int64, device=self.device)
        scratch = torch.empty(max(8 * self.n_blocks, 8), dtype=torch.uint8, device=self.device)
        check(lib().lz_verify(self.h, _ptr(out), _ptr(tree), _ptr(scratch), scratch.numel(),
                              _stream(stream)))
        return tree

    def verify_range(self, out: torch.Tensor, offset: int, length: int,
                     scratch: torch.Tensor | None = None, stream=None) -> None:
        """lz_verify_range: every block of x[offset, offset+length), decoded at
        out, against its source hash (a mismatch surfaces in sync_status)."""
        B = 1 << int(self.info.block_log2)
        need = max(8, 8 * (-(-length // B)))
        if scratch is None or scratch.numel() < need:
            scratch = torch.empty(need, dtype=torch.uint8, device=self.device)
        check(lib().lz_verify_range(self.h, _ptr(out), offset, length, _ptr(scratch), scratch.numel(),
                                    _stream(stream)))

    def last_stats(self, stream=None) -> _lib.Stats:
        """lz_last_stats: blocks decoded by the last request call (covering
        blocks plus dependency closure), scratch slots, covering pairs."""
        st = _lib.Stats()
        check(lib().lz_last_stats(self.h, C.byref(st), _stream(stream)))
        return st

    def sync_status(self, stream=None) -> None:
        check(lib().lz_sync_status(self.h, _stream(stream)))


def encode_split(data, **params) -> bytes:
    """Stream-separated FASTQ container of host bytes (lz_encode_split): the
    id, sequence, '+' and quality lines as four archives of this codec plus a
    read index.  Keyword arguments override lz_params fields (kind is 0)."""
    if isinstance(data, np.ndarray):
        a = np.ascontiguousarray(data, dtype=np.uint8)
    else:
        a = np.frombuffer(memoryview(data), dtype=np.uint8)
    p = _lib.default_params(**params)
    out = C.c_void_p()
    n = C.c_uint64()
    check(lib().lz_encode_split(C.c_void_p(a.ctypes.data if a.size else 0), a.size, C.byref(p),
                                C.byref(out), C.byref(n)))
    try:
        return bytes(memoryview((C.c_char * n.value).from_address(out.value)))
    finally:
        lib().lz_free(out)


class SplitArchive:
    """A stream-separated FASTQ container resident in HBM (lz_split_open):
    whole-file decode, byte ranges and read lookups of the original file."""

    def __init__(self, container, device: str | torch.device = "cuda:0", stream=None):
        self.device = torch.device(device)
        if isinstance(container, torch.Tensor):
            assert container.dtype == torch.uint8 and container.is_cuda and container.is_contiguous()
            self.d_archive = container
        else:
            host = torch.from_numpy(np.frombuffer(memoryview(container), dtype=np.uint8).copy())
            self.d_archive = torch.empty(host.numel(), dtype=torch.uint8, device=self.device)
            self.d_archive.copy_(host)
        i = _lib.SplitInfo()
        check(lib().lz_split_info_get(_ptr(self.d_archive), self.d_archive.numel(), _stream(stream),
                                      C.byref(i)))
        self.info = i
        self.ws = torch.empty(max(i.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        self.h = C.c_void_p()
        check(lib().lz_split_open(_ptr(self.d_archive), self.d_archive.numel(), _ptr(self.ws),
                                  self.ws.numel(), _stream(stream), C.byref(self.h)))

    @property
    def n(self) -> int:
        return int(self.info.n)

    @property
    def n_reads(self) -> int:
        return int(self.info.n_reads)

    def close(self):
        if self.h:
            lib().lz_split_close(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream_handle(self, k: int) -> C.c_void_p:
        h = C.c_void_p()
        check(lib().lz_split_stream(self.h, k, C.byref(h)))
        return h

    def set_tuning(self, sync_mode: int | None = None, wg_per_cu: int | None = None):
        for k in range(4):
            h = self.stream_handle(k)
            t = _lib.Tuning()
            check(lib().lz_get_tuning(h, C.byref(t)))
            if sync_mode is not None:
                t.sync_mode = sync_mode
            if wg_per_cu is not None:
                t.wg_per_cu = wg_per_cu
            check(lib().lz_set_tuning(h, C.byref(t)))

    def scratch_bytes(self, n_requests: int) -> int:
        b = C.c_uint64()
        check(lib().lz_split_scratch_bytes(self.h, max(1, n_requests), C.byref(b)))
        return int(b.value)

    def decode_all(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(self.n, 1), dtype=torch.uint8, device=self.device)
        check(lib().lz_split_decode_all(self.h, _ptr(out), out.numel(), _stream(stream)))
        return out[: self.n]

    def decode_range(self, offset: int, length: int, out: torch.Tensor | None = None,
                     scratch: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(length, 1), dtype=torch.uint8, device=self.device)
        if scratch is None:
            scratch = torch.empty(self.scratch_bytes(1), dtype=torch.uint8, device=self.device)
        check(lib().lz_split_decode_range(self.h, offset, length, _ptr(out), _ptr(scratch),
                                          scratch.numel(), _stream(stream)))
        return out[:length]

    def read_lookup(self, ids, out: torch.Tensor | None = None, offsets: torch.Tensor | None = None,
                    scratch: torch.Tensor | None = None, stream=None):
        ids = torch.as_tensor(ids, dtype=torch.int64, device=self.device).contiguous()
        n = ids.numel()
        if out is None:
            out = torch.empty(max(1, n * int(self.info.max_record_len)), dtype=torch.uint8, device=self.device)
        if offsets is None:
            offsets = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        if scratch is None:
            scratch = torch.empty(self.scratch_bytes(n), dtype=torch.uint8, device=self.device)
        check(lib().lz_split_read_lookup(self.h, _ptr(ids), n, _ptr(out), out.numel(), _ptr(offsets),
                                         _ptr(scratch), scratch.numel(), _stream(stream)))
        return out, offsets

    def sync_status(self, stream=None) -> None:
        check(lib().lz_split_sync_status(self.h, _stream(stream)))
