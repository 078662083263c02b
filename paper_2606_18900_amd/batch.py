"""Batched random access: many uneven read/range requests resolved together by
one lz_decode_batch launch sequence (closure over all requests, one decode
launch over the shared level-ordered block queue, gather), captured once in a
HIP graph and replayed with new request contents."""
from __future__ import annotations

import numpy as np
import torch

READ, RANGE = 0, 1


class Batcher:
    """Fixed-capacity request batch on one Archive.

    submit(kind, a, b) copies up to n_max requests (kind 0: read id a; kind 1:
    bytes [a, a+b)) into fixed device buffers and replays the captured graph
    (or launches eagerly when use_graph is False).  Results stay on the device
    until `results()` / `result(k)` read them."""

    def __init__(self, arc, n_max: int, out_cap: int, n_slots: int | None = None,
                 use_graph: bool = True, stream: torch.cuda.Stream | None = None,
                 scratch: torch.Tensor | None = None):
        self.arc = arc
        self.n_max = int(n_max)
        dev = arc.device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self.reqs = torch.zeros((self.n_max, 3), dtype=torch.int64, device=dev)
        self.n = torch.zeros(1, dtype=torch.int32, device=dev)
        self.out = torch.empty(max(1, out_cap), dtype=torch.uint8, device=dev)
        self.offsets = torch.zeros(self.n_max + 1, dtype=torch.int64, device=dev)
        # scratch may be shared by Batchers whose batches run on one stream
        need = arc.scratch_bytes(self.n_max, n_slots)
        if scratch is None:
            scratch = torch.empty(need, dtype=torch.uint8, device=dev)
        assert scratch.numel() >= need
        self.scratch = scratch
        self.h_reqs = torch.zeros((self.n_max, 3), dtype=torch.int64).pin_memory()
        self.h_n = torch.zeros(1, dtype=torch.int32).pin_memory()
        self.count = 0
        self.graph = None
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        self._launch()                       # eager once: initialises everything
        self.stream.synchronize()
        if use_graph:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self._launch()
            self.graph = g

    def _launch(self):
        self.arc.decode_batch(self.reqs, self.n, self.n_max, self.out, self.offsets,
                              self.scratch, stream=self.stream)

    def submit(self, kind, a, b) -> None:
        kind = np.asarray(kind, dtype=np.int64)
        k = int(kind.shape[0])
        if k > self.n_max:
            raise ValueError("batch of %d exceeds capacity %d" % (k, self.n_max))
        hr = self.h_reqs.numpy()
        hr[:k, 0] = kind
        hr[:k, 1] = np.asarray(a, dtype=np.int64)
        hr[:k, 2] = np.asarray(b, dtype=np.int64)
        self.h_n.numpy()[0] = k
        with torch.cuda.stream(self.stream):
            self.reqs[:k].copy_(self.h_reqs[:k], non_blocking=True)
            self.n.copy_(self.h_n, non_blocking=True)
        self.count = k
        if self.graph is not None:
            with torch.cuda.stream(self.stream):
                self.graph.replay()
        else:
            self._launch()

    def event(self, timing: bool = False) -> torch.cuda.Event:
        e = torch.cuda.Event(enable_timing=timing)
        e.record(self.stream)
        return e

    def synchronize(self) -> None:
        self.stream.synchronize()
        self.arc.sync_status(stream=self.stream)

    def results(self) -> list[bytes]:
        self.synchronize()
        o = self.offsets[: self.count + 1].cpu().numpy()
        data = self.out[: int(o[-1])].cpu().numpy().tobytes() if self.count else b""
        return [data[int(o[i]):int(o[i + 1])] for i in range(self.count)]
