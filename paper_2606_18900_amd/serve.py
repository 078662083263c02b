"""Served decode loop: an open-loop request stream over resident archives.

Requests (read lookups and byte ranges) arrive on a schedule; the loop admits
them as their arrival time passes and serves them with continuous batching.
Every archive has several batch lanes; a lane owns a HIP stream, a handle of
its own on the archive (so its workspace serves only that lane), an output
window, request tables and a scratch area for dependency closures, and one
captured lz_decode_batch graph.  Whenever a lane is free the oldest pending
work of its archive is packed into its next batch (up to n_max requests and
`window` output bytes) and launched on the lane's stream, so batches of
different lanes run on the device at the same time while the host packs the
next ones.

Admission by device-memory budget: all device memory of the lanes (windows,
tables, scratch, workspaces) is reserved up front and must fit the budget
(ValueError otherwise); a request is admitted into the queue of its archive
when it arrives and enters a batch when a lane frees up.  A range longer than
the window is served window by window; a read whose record does not fit one
window can never be served within the budget and is refused with LZ_EBUDGET.
A loop that makes no progress for `stall_s` seconds raises instead of waiting
forever.  Latency of a request = the time its last window is seen complete
minus its scheduled arrival (queueing included).

Decoding happens in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from ._lib import LZ_EBUDGET, NAMES
from .batch import Batcher

READ, RANGE = 0, 1


class Server:
    """Continuous-batching server over one or more Archives.

    archives: list of Archive (FASTQ archives serve reads; any serves ranges)
    read_starts: per archive, the host copy of its read index (u64 record
        starts, n_reads + 1 entries) or None; used to size read outputs
    budget: device bytes the lanes may hold in total
    lanes: batch lanes (batches in flight at once) per archive; n_max:
        requests per batch; window: output bytes per batch
    use_graph: replay a captured graph per batch (False: eager launches)
    batcher: lane factory (Batcher; a stand-in with the same interface can
        replace it to exercise the scheduling on the host)
    """

    def __init__(self, archives, read_starts, budget: int = 16 << 30, lanes: int = 4,
                 n_max: int = 1024, window: int = 256 << 20, use_graph: bool = True,
                 keep_results: bool = False, batcher=Batcher, stall_s: float = 30.0):
        self.archives = list(archives)
        self.starts = list(read_starts)
        self.n_max = int(n_max)
        self.window = int(window)
        self.keep = keep_results
        self.stall_s = stall_s
        real = batcher is Batcher
        per_archive = []
        for arc, st in zip(self.archives, self.starts):
            slots = arc.n_blocks
            ws = int(arc.info.workspace_bytes) if real else 0
            per_archive.append(self.window + 16 * (self.n_max + 1) + arc.scratch_bytes(self.n_max, slots) + ws)
        need = lanes * sum(per_archive)
        if need > budget:
            raise ValueError("budget %d below the lanes' windows, tables, scratch and workspaces (%d)"
                             % (budget, need))
        self.device_bytes = need
        self.lanes = []
        for arc in self.archives:
            lane = []
            for _ in range(lanes):
                if real:
                    import torch
                    from .archive import Archive
                    h = Archive(arc.d_archive, device=arc.device)     # own workspace
                    h.set_tuning(**{f: getattr(arc.tuning(), f) for f in ("sync_mode", "wg_per_cu", "req_sync_mode", "plan_blocks")})
                    lane.append(batcher(h, self.n_max, self.window, n_slots=arc.n_blocks,
                                        use_graph=use_graph, stream=torch.cuda.Stream(device=arc.device)))
                else:
                    lane.append(batcher(arc, self.n_max, self.window, n_slots=arc.n_blocks,
                                        use_graph=use_graph))
            self.lanes.append(lane)
        self.stamps = []     # (archive, lane, start event, end event, request ids) per batch

    def _request_bytes(self, arch, kind, a, b):
        if kind == READ:
            s = self.starts[arch]
            return int(s[a + 1] - s[a])
        return int(b)

    def run(self, trace: dict, time_limit_s: float | None = None) -> dict:
        """Serve `trace` (arrays t [s], archive, kind, a, b as made by
        gen.requests.poisson_trace).  Returns latency percentiles (ms),
        completed and refused counts, throughput, device overlap of the
        batches and, with keep_results, the outputs."""
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
        refused = {}
        results = {} if self.keep else None
        free = [list(range(len(l))) for l in self.lanes]
        inflight = []                               # (archive, lane, event, entries)
        self.stamps = []
        i = 0
        settled = 0                                 # completed or refused
        t0 = time.perf_counter()
        last_progress = t0
        limit = None if time_limit_s is None else t0 + time_limit_s
        while settled < n:
            now = time.perf_counter()
            if limit is not None and now > limit:
                break
            rel = now - t0
            # admit every request whose arrival time has passed
            while i < n and t_arr[i] <= rel:
                k = int(arch[i])
                if kind[i] == READ:
                    nb = self._request_bytes(k, READ, int(ra[i]), 0)
                    if nb > self.window:            # never fits a lane's window
                        refused[i] = LZ_EBUDGET
                        settled += 1
                    else:
                        pending[k].append((i, READ, int(ra[i]), 0, nb))
                        left[i] = 1
                        out_bytes[i] = nb
                else:
                    off, ln = int(ra[i]), int(rb[i])
                    pieces = max(1, -(-ln // self.window))
                    left[i] = pieces
                    out_bytes[i] = ln
                    for p in range(pieces):
                        w = min(self.window, ln - p * self.window)
                        pending[k].append((i, RANGE, off + p * self.window, w, w))
                i += 1
                last_progress = now
            # completions
            still = []
            for k, ln, ev, entries in inflight:
                if ev.query():
                    tc = time.perf_counter() - t0
                    if self.keep:                   # pieces complete in any order across lanes
                        got = self.lanes[k][ln].results()
                        for (rid, _, off, _, _), g in zip(entries, got):
                            results.setdefault(rid, []).append((off, g))
                    for rid, _, _, _, _ in entries:
                        left[rid] -= 1
                        if left[rid] == 0:
                            done_t[rid] = tc
                            settled += 1
                    free[k].append(ln)
                    last_progress = time.perf_counter()
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
                    if not entries:                 # admission guarantees every piece fits
                        raise RuntimeError("pending entry larger than the window")
                    ln = free[k].pop()
                    bt = self.lanes[k][ln]
                    start = bt.event(True)
                    bt.submit([e[1] for e in entries], [e[2] for e in entries], [e[3] for e in entries])
                    end = bt.event(True)
                    self.stamps.append((k, ln, start, end, [e[0] for e in entries]))
                    inflight.append((k, ln, end, entries))
                    launched = True
                    last_progress = time.perf_counter()
            if launched:
                continue
            if not inflight and i < n and not any(pending):
                # idle until the next arrival
                wait = t_arr[i] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
                last_progress = time.perf_counter()
            elif time.perf_counter() - last_progress > self.stall_s:
                raise RuntimeError("served decode loop made no progress for %.0f s" % self.stall_s)
        for lane in self.lanes:
            for bt in lane:
                bt.synchronize()
        wall = time.perf_counter() - t0
        ok = ~np.isnan(done_t)
        lat = (done_t[ok] - t_arr[ok]) * 1e3
        res = {
            "offered": n,
            "completed": int(ok.sum()),
            "refused": {NAMES[c]: sum(1 for v in refused.values() if v == c) for c in set(refused.values())},
            "wall_s": round(wall, 3),
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "served_req_per_s": round(float(ok.sum()) / wall, 1),
            "served_GB_per_s": round(float(out_bytes[ok].sum()) / wall / 1e9, 3),
            "device_overlap": self.overlap(),
        }
        if self.keep:
            res["results"] = {rid: b"".join(g for _, g in sorted(v, key=lambda p: p[0]))
                              for rid, v in results.items()}
            res["refused_ids"] = dict(refused)
        return res

    def intervals(self):
        """Device [start, end] of every batch of the last run, in ms from the
        first batch's start (HIP events recorded on the lanes' streams)."""
        if not self.stamps or not hasattr(self.stamps[0][2], "elapsed_time"):
            return []
        ref = self.stamps[0][2]
        return [(k, ln, ref.elapsed_time(s), ref.elapsed_time(e), rids)
                for k, ln, s, e, rids in self.stamps]

    def overlap(self):
        """Batches that started on the device while another batch was still
        running, and the largest number running at once."""
        iv = self.intervals()
        if not iv:
            return None
        ev = sorted([(s, 1) for _, _, s, _, _ in iv] + [(e, -1) for _, _, _, e, _ in iv],
                    key=lambda p: (p[0], p[1]))
        cur = peak = 0
        for _, d in ev:
            cur += d
            peak = max(peak, cur)
        started_inside = sum(1 for a in iv if any(b is not a and b[2] < a[2] < b[3] for b in iv))
        return {"batches": len(iv), "started_while_another_ran": started_inside, "max_concurrent": peak}
