"""Served decode loop: an open-loop request stream over resident archives.

Requests (read lookups and byte ranges) arrive on a schedule; the loop admits
them as their arrival time passes and serves them with continuous batching:
every archive has a few batch lanes (one captured lz_decode_batch graph and
fixed buffers each), and whenever a lane is free the oldest pending work of
that archive is packed into its next batch (up to n_max requests and `window`
output bytes).  All lanes feed one HIP stream: batches run back to back in
submission order while the host packs the ones behind them, and calls on an
archive handle (whose workspace one call uses at a time) never overlap.  A range longer than the window is
served window by window, each window a batch entry, so every batch's output
fits its lane's buffer.  All device memory of the lanes (outputs, scratch
slots for dependency closures, request tables) is allocated up front and must
fit the memory budget; an archive's scratch has a slot for every block, so no
batch can fail for capacity.  Latency of a request = the time its last window
is seen complete minus its scheduled arrival (queueing included).

Decoding happens in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from .batch import Batcher

READ, RANGE = 0, 1


class Server:
    """Continuous-batching server over one or more Archives.

    archives: list of Archive (FASTQ archives serve reads; any serves ranges)
    read_starts: per archive, the host copy of its read index (u64 record
        starts, n_reads + 1 entries) or None; used to size read outputs
    budget: device bytes the lanes may hold in total
    lanes: batch lanes (batches in flight) per archive; n_max: requests per batch
    window: output bytes per batch (ranges are cut into window-sized pieces)
    use_graph: replay a captured graph per batch (False: eager launches)
    batcher: lane factory (Batcher; a stand-in with the same interface can
        replace it to exercise the scheduling on the host)
    """

    def __init__(self, archives, read_starts, budget: int = 16 << 30, lanes: int = 4,
                 n_max: int = 1024, window: int = 256 << 20, use_graph: bool = True,
                 keep_results: bool = False, batcher=Batcher):
        self.archives = list(archives)
        self.starts = list(read_starts)
        self.stream = None
        if batcher is Batcher:
            import torch
            self.stream = torch.cuda.Stream(device=self.archives[0].device)
        self.n_max = int(n_max)
        self.window = int(window)
        self.keep = keep_results
        B = [1 << int(a.info.block_log2) for a in self.archives]
        # every lane owns an output window and request tables; the lanes of an
        # archive share one scratch area (their batches run one after another
        # on the stream) with a slot for every block, enough for any closure
        per_lane = [self.window + 64 * (self.n_max + 1) for _ in self.archives]
        scratch = [a.scratch_bytes(self.n_max, a.n_blocks) for a in self.archives]
        need = lanes * sum(per_lane) + sum(scratch)
        if need > budget:
            raise ValueError("budget %d below the lanes' windows and scratch (%d)" % (budget, need))
        self.lanes = []
        self.device_bytes = need
        for k, arc in enumerate(self.archives):
            # the lanes of an archive share its handle and one stream: their
            # batches run in submission order, so calls on the handle never
            # overlap, while the host packs the next batches ahead
            stream = self.stream if batcher is Batcher else None
            shared = None
            if batcher is Batcher:
                import torch
                shared = torch.empty(scratch[k], dtype=torch.uint8, device=arc.device)
            lane = [batcher(arc, self.n_max, self.window, n_slots=arc.n_blocks, use_graph=use_graph,
                            stream=stream, scratch=shared)
                    for _ in range(lanes)]
            self.lanes.append(lane)
        assert self.device_bytes <= budget

    def _request_bytes(self, arch, kind, a, b):
        if kind == READ:
            s = self.starts[arch]
            return int(s[a + 1] - s[a])
        return int(b)

    def run(self, trace: dict, time_limit_s: float | None = None) -> dict:
        """Serve `trace` (arrays t [s], archive, kind, a, b as made by
        gen.requests.poisson_trace).  Returns latency percentiles (ms),
        completed count, throughput and, with keep_results, the outputs."""
        t_arr = np.asarray(trace["t"], dtype=np.float64)
        arch = np.asarray(trace["archive"], dtype=np.int64)
        kind = np.asarray(trace["kind"], dtype=np.int64)
        ra = np.asarray(trace["a"], dtype=np.int64)
        rb = np.asarray(trace["b"], dtype=np.int64)
        n = len(t_arr)
        pending = [collections.deque() for _ in self.archives]
        left = np.zeros(n, dtype=np.int64)          # windows not yet completed
        done_t = np.full(n, np.nan)
        out_bytes = np.zeros(n, dtype=np.int64)
        results = {} if self.keep else None
        free = [list(range(len(l))) for l in self.lanes]
        inflight = []                               # (archive, lane, event, entries)
        i = 0
        completed = 0
        t0 = time.perf_counter()
        limit = None if time_limit_s is None else t0 + time_limit_s
        while completed < n:
            now = time.perf_counter()
            if limit is not None and now > limit:
                break
            rel = now - t0
            # admit every request whose arrival time has passed
            while i < n and t_arr[i] <= rel:
                k = int(arch[i])
                if kind[i] == READ:
                    pending[k].append((i, READ, int(ra[i]), 0, self._request_bytes(k, READ, int(ra[i]), 0)))
                    left[i] = 1
                    out_bytes[i] = pending[k][-1][4]
                else:
                    off, ln = int(ra[i]), int(rb[i])
                    pieces = max(1, -(-ln // self.window))
                    left[i] = pieces
                    out_bytes[i] = ln
                    for p in range(pieces):
                        w = min(self.window, ln - p * self.window)
                        pending[k].append((i, RANGE, off + p * self.window, w, w))
                i += 1
            # completions
            still = []
            for k, ln, ev, entries in inflight:
                if ev.query():
                    tc = time.perf_counter() - t0
                    if self.keep:
                        got = self.lanes[k][ln].results()
                        for (rid, _, _, _, _), g in zip(entries, got):
                            results.setdefault(rid, []).append(g)
                    for rid, _, _, _, _ in entries:
                        left[rid] -= 1
                        if left[rid] == 0:
                            done_t[rid] = tc
                            completed += 1
                    free[k].append(ln)
                else:
                    still.append((k, ln, ev, entries))
            inflight = still
            # launch: every free lane takes the oldest pending work of its archive
            launched = False
            for k in range(len(self.archives)):
                while free[k] and pending[k]:
                    entries, total = [], 0
                    q = pending[k]
                    while q and len(entries) < self.n_max and total + q[0][4] <= self.window:
                        e = q.popleft()
                        entries.append(e)
                        total += e[4]
                    ln = free[k].pop()
                    bt = self.lanes[k][ln]
                    bt.submit([e[1] for e in entries], [e[2] for e in entries], [e[3] for e in entries])
                    inflight.append((k, ln, bt.event(), entries))
                    launched = True
            if not launched and not inflight and i < n and not any(pending):
                # idle until the next arrival
                wait = t_arr[i] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        for lane in self.lanes:
            for bt in lane:
                bt.synchronize()
        wall = time.perf_counter() - t0
        ok = ~np.isnan(done_t)
        lat = (done_t[ok] - t_arr[ok]) * 1e3
        res = {
            "offered": n,
            "completed": int(ok.sum()),
            "wall_s": round(wall, 3),
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "served_req_per_s": round(float(ok.sum()) / wall, 1),
            "served_GB_per_s": round(float(out_bytes[ok].sum()) / wall / 1e9, 3),
        }
        if self.keep:
            res["results"] = {rid: b"".join(v) for rid, v in results.items()}
        return res
