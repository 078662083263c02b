"""The library's kernels run on the CPU (tests/emu: the HIP language and
runtime replaced by a host shim, every work-item a host thread, wave
operations as rendezvous of the wave's 64 lanes), under AddressSanitizer and
UBSan.  Each case decodes an archive through the C ABI -- whole file, three
byte ranges and, for FASTQ, four reads -- and must reproduce the source.  A
wave operation reached by only part of a wave, a lane that leaves a wave
while others wait in a wave operation, or a wait that does not end, stops the
run: on gfx950 those would make results depend on how the compiler laid out
the branch, or hang.  (Found this way and fixed: the one-workgroup request
planner let waves read the closure list's length at different times within a
round, so they could leave its loop in different rounds.)"""
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

CASES = {
    # FASTQ with 1 KiB blocks: literal groups, short streams, in-block chains, reads
    "fastq_1k": ("fastq", dict(kind=1, block_log2=10, min_match=16, hash_len=16, hash_bits=16, max_level=16,
                               level_penalty=4, lit_lanes=64, seq_lanes=16)),
    # FASTQ with 16 KiB blocks and the default lane counts (the benchmark's profile)
    "fastq_16k": ("fastq16", dict(kind=1, level_penalty=32)),
    # 64-byte blocks, deep dependency levels, self-overlapping matches
    "deep_64": ("motifs", dict(block_log2=6, min_match=4, hash_len=4, hash_bits=14, max_level=64,
                               level_penalty=0, lit_lanes=16, seq_lanes=4)),
}


def _data(kind):
    from gen.fastq import fastq
    if kind == "fastq":
        x, _ = fastq(n_records=60, seed=6)
        return bytes(x)
    if kind == "fastq16":
        x, _ = fastq(n_records=80, seed=7)
        return bytes(x)
    rng = np.random.default_rng(3)
    motifs = [rng.integers(65, 70, 50, dtype=np.uint8).tobytes() for _ in range(6)]
    s = bytearray()
    while len(s) < 4000:
        s += motifs[int(rng.integers(0, 6))] if rng.random() < 0.6 else \
            rng.integers(65, 91, int(rng.integers(1, 40)), dtype=np.uint8).tobytes()
    return bytes(s[:4000])


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    import shutil
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    import build as emu_build
    return emu_build.build(str(tmp_path_factory.mktemp("emu")))


def test_kernels_under_lockstep_emulation(emu, orc, tmp_path):
    procs = {}
    for name, (kind, params) in CASES.items():
        x = _data(kind)
        a = orc.encode(x, **params)
        (tmp_path / (name + ".lz")).write_bytes(a)
        (tmp_path / (name + ".src")).write_bytes(x)
        env = dict(os.environ, LZ_EMU_LIMIT_S="60", ASAN_OPTIONS="detect_leaks=1")
        procs[name] = subprocess.Popen([emu, str(tmp_path / (name + ".lz")), str(tmp_path / (name + ".src"))],
                                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env)
    fails = []
    for name, p in procs.items():
        try:
            out, err = p.communicate(timeout=600)
        except subprocess.TimeoutExpired:
            p.kill()
            out, err = p.communicate()
            fails.append("%s: timed out" % name)
            continue
        if p.returncode != 0 or b"emu ok" not in out:
            fails.append("%s: rc %d\n%s\n%s" % (name, p.returncode, out.decode(errors="replace")[-500:],
                                              err.decode(errors="replace")[-3000:]))
    assert not fails, "\n".join(fails)
