"""Autotuner: launch settings of one archive on one device, and the rANS lane
counts of an encoding.

Whole-file decode (`tune`): the decode kernel's synchronisation mode (one
launch per dependency level, or one cooperative launch with a grid barrier
between levels) and the workgroups per CU of its grid (1..3: the kernel's
launch bounds and its 52 KB of LDS hold three workgroups per CU, so more only
queue).  Every candidate decodes the archive into the same buffer and must
reproduce the archive's source FNV tree (device hash of the output), so a
faster but wrong setting can never win.

Request calls (`tune_requests`): the closure decode's synchronisation mode
and the size up to which a call is planned by one workgroup in one launch
instead of the eight-kernel path.  The workload is one single read and one
batch of 256 reads; every candidate's bytes must equal those of the default
setting.

Encoding (`tune_encoding`): the literal and sequence rANS lane counts are
fixed when a file is encoded, so they are tuned by re-encoding a sample with
each candidate, decoding it on the device (verified by the source hash) and
keeping the fastest decode whose ratio is within `max_ratio_loss` of the
best.  The LDS tile is not a knob: one 16 KiB block per 256-thread workgroup
is the shape whose 52 KB of LDS fits three workgroups per CU; a tile of two
blocks needs twice the LDS and halves the resident workgroups.

The median of `reps` timed runs (HIP events on the stream) ranks candidates.
`tune` and `tune_requests` cache their result in a JSON file keyed by device
name, archive size, block count, level count and source hash."""
from __future__ import annotations

import json
import os

import numpy as np
import torch

MODES = (0, 1)
WG_PER_CU = (1, 2, 3)
REQ_MODES = (0, 1)
PLAN_BLOCKS = (1, 4096, 65536)       # 1: never one-workgroup planning
LANES = ((256, 64), (128, 64), (128, 32), (64, 32))


def _key(arc, what: str = "decode") -> str:
    i = arc.info
    dev = torch.cuda.get_device_name(arc.device)
    return "%s|%s|n=%d|blocks=%d|levels=%d|fnv=%016x" % (what, dev, i.n, i.n_blocks, i.n_levels,
                                                         int(i.source_fnv) & (2 ** 64 - 1))


def _load(cache_path):
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            return json.load(f)
    return {}


def _store(cache_path, cache):
    if not cache_path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)


def _median_ms(fn, reps: int, stream) -> float:
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def tune(arc, cache_path: str | None = None, reps: int = 5, out: torch.Tensor | None = None,
         modes=MODES, wg_per_cu=WG_PER_CU) -> dict:
    """Pick and apply the fastest verified (sync_mode, wg_per_cu) for whole-file
    decodes of `arc`.  Returns {"sync_mode", "wg_per_cu", "ms", "table"
    (all candidates), "cached"}."""
    key = _key(arc)
    cache = _load(cache_path)
    if key in cache:
        best = cache[key]
        arc.set_tuning(sync_mode=best["sync_mode"], wg_per_cu=best["wg_per_cu"])
        return dict(best, cached=True)
    if out is None:
        out = torch.empty(arc.n + 256, dtype=torch.uint8, device=arc.device)
    want = int(arc.info.source_fnv) & (2 ** 64 - 1)
    stream = torch.cuda.current_stream(arc.device)
    table = []
    for mode in modes:
        for wg in wg_per_cu:
            arc.set_tuning(sync_mode=mode, wg_per_cu=wg)
            out.fill_(0)
            arc.decode_all(out)
            tree = int(arc.verify(out).cpu().item()) & (2 ** 64 - 1)
            arc.sync_status()
            if tree != want:
                table.append({"sync_mode": mode, "wg_per_cu": wg, "ms": None, "ok": False})
                continue
            ms = _median_ms(lambda: arc.decode_all(out), reps, stream)
            arc.sync_status()
            table.append({"sync_mode": mode, "wg_per_cu": wg, "ms": ms, "ok": True})
    good = [r for r in table if r["ok"]]
    if not good:
        raise RuntimeError("no launch setting reproduced the archive's source hash")
    best = min(good, key=lambda r: r["ms"])
    arc.set_tuning(sync_mode=best["sync_mode"], wg_per_cu=best["wg_per_cu"])
    res = {"sync_mode": best["sync_mode"], "wg_per_cu": best["wg_per_cu"], "ms": best["ms"], "table": table}
    cache[key] = res
    _store(cache_path, cache)
    return dict(res, cached=False)


def tune_requests(arc, cache_path: str | None = None, reps: int = 20, seed: int = 0,
                  modes=REQ_MODES, plan_blocks=PLAN_BLOCKS) -> dict:
    """Pick and apply the fastest (req_sync_mode, plan_blocks) for read
    lookups on `arc` (a FASTQ archive): the time of one single read plus one
    batch of 256 reads, medians of `reps`.  Every candidate's output must
    equal the default setting's.  Returns {"req_sync_mode", "plan_blocks",
    "us", "table", "cached"}."""
    key = _key(arc, "requests")
    cache = _load(cache_path)
    if key in cache:
        best = cache[key]
        arc.set_tuning(req_sync_mode=best["req_sync_mode"], plan_blocks=best["plan_blocks"])
        return dict(best, cached=True)
    dev = arc.device
    rng = np.random.default_rng(seed)
    one = torch.tensor([int(rng.integers(0, arc.n_reads))], dtype=torch.int64, device=dev)
    many = torch.tensor(rng.integers(0, arc.n_reads, 256), dtype=torch.int64, device=dev)
    cap = 256 * int(arc.info.max_record_len)
    out1 = torch.empty(cap, dtype=torch.uint8, device=dev)
    outn = torch.empty(cap, dtype=torch.uint8, device=dev)
    off1 = torch.empty(2, dtype=torch.int64, device=dev)
    offn = torch.empty(257, dtype=torch.int64, device=dev)
    sc = torch.empty(arc.scratch_bytes(256), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def run_both():
        arc.read_lookup(one, out=out1, offsets=off1, scratch=sc)
        arc.read_lookup(many, out=outn, offsets=offn, scratch=sc)

    arc.set_tuning(req_sync_mode=0, plan_blocks=4096)
    run_both()
    torch.cuda.synchronize()
    arc.sync_status()
    ref = (out1[: int(off1[1])].clone(), outn[: int(offn[256])].clone())
    table = []
    for mode in modes:
        for pb in plan_blocks:
            arc.set_tuning(req_sync_mode=mode, plan_blocks=pb)
            out1.fill_(0)
            outn.fill_(0)
            run_both()
            torch.cuda.synchronize()
            arc.sync_status()
            ok = torch.equal(out1[: int(off1[1])], ref[0]) and torch.equal(outn[: int(offn[256])], ref[1])
            if not ok:
                table.append({"req_sync_mode": mode, "plan_blocks": pb, "us": None, "ok": False})
                continue
            us1 = 1e3 * _median_ms(lambda: arc.read_lookup(one, out=out1, offsets=off1, scratch=sc), reps, stream)
            usn = 1e3 * _median_ms(lambda: arc.read_lookup(many, out=outn, offsets=offn, scratch=sc), reps, stream)
            arc.sync_status()
            table.append({"req_sync_mode": mode, "plan_blocks": pb, "single_us": us1, "batch256_us": usn,
                          "us": us1 + usn, "ok": True})
    good = [r for r in table if r["ok"]]
    if not good:
        raise RuntimeError("no request setting reproduced the default setting's output")
    best = min(good, key=lambda r: r["us"])
    arc.set_tuning(req_sync_mode=best["req_sync_mode"], plan_blocks=best["plan_blocks"])
    res = {"req_sync_mode": best["req_sync_mode"], "plan_blocks": best["plan_blocks"], "us": best["us"],
           "table": table}
    cache[key] = res
    _store(cache_path, cache)
    return dict(res, cached=False)


def tune_encoding(sample: bytes, params: dict, device="cuda:0", lanes=LANES, reps: int = 5,
                  max_ratio_loss: float = 0.01) -> dict:
    """Re-encode `sample` with every (lit_lanes, seq_lanes) candidate and time
    its whole-file decode (verified by the source hash).  Returns the fastest
    candidate whose ratio is within max_ratio_loss of the best ratio, and the
    table {"lit_lanes", "seq_lanes", "ratio", "ms", "gbps", "ok"}."""
    from .archive import Archive, encode
    dev = torch.device(device)
    table = []
    out = None
    for lit, seq in lanes:
        p = dict(params, lit_lanes=lit, seq_lanes=seq)
        a = encode(sample, **p)
        arc = Archive(a, device=dev)
        if out is None or out.numel() < arc.n + 256:
            out = torch.empty(arc.n + 256, dtype=torch.uint8, device=dev)
        arc.decode_all(out)
        tree = int(arc.verify(out).cpu().item()) & (2 ** 64 - 1)
        arc.sync_status()
        ok = tree == int(arc.info.source_fnv) & (2 ** 64 - 1)
        ms = _median_ms(lambda: arc.decode_all(out), reps, torch.cuda.current_stream(dev)) if ok else None
        arc.sync_status()
        table.append({"lit_lanes": lit, "seq_lanes": seq, "ratio": len(sample) / len(a), "ms": ms,
                      "gbps": len(sample) / ms / 1e6 if ms else None, "ok": ok})
        arc.close()
    good = [r for r in table if r["ok"]]
    if not good:
        raise RuntimeError("no lane setting reproduced the sample's source hash")
    top = max(r["ratio"] for r in good)
    near = [r for r in good if r["ratio"] >= top * (1 - max_ratio_loss)]
    best = min(near, key=lambda r: r["ms"])
    return {"lit_lanes": best["lit_lanes"], "seq_lanes": best["seq_lanes"], "ratio": best["ratio"],
            "ms": best["ms"], "table": table}
