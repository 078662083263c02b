"""Build liblz.so in-tree with hipcc for gfx950 (no JIT, no torch extension)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblz.so")
LIB_CLK = os.path.join(HERE, "liblz_clk.so")   # instrumented variant (stage clocks)
SOURCES = ["kernels.hip", "noalloc.hip", "split.hip", "runtime.cpp", "encode.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INC, "-I", CSRC]


def build(verbose: bool = False, stage_clocks: bool = False) -> str:
    """Build liblz.so; with stage_clocks, the instrumented variant
    liblz_clk.so (per-stage cycle counters of the decode kernel)."""
    objs = []
    bdir = os.path.join(HERE, "_build_clk" if stage_clocks else "_build")
    lib = LIB_CLK if stage_clocks else LIB
    extra = ["-DLZ_STAGE_CLOCKS"] if stage_clocks else []
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for s in SOURCES:
        o = os.path.join(bdir, s + ".o")
        cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(o)
    fail = []
    for s, p in procs:
        out, _ = p.communicate()
        if out and (verbose or p.returncode):
            sys.stdout.write(out.decode(errors="replace"))
        if p.returncode:
            fail.append(s)
    if fail:
        raise RuntimeError("hipcc failed on " + ", ".join(fail))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, stage_clocks="--stage-clocks" in sys.argv))
