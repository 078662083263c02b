"""Build the CPU emulation of liblz (test harness only): the library's own
sources, compiled for the host with the shim in tests/emu/shim standing in
for HIP, under AddressSanitizer and UBSan, plus the driver emu_main.cpp.
-O0 keeps each wave operation at one place in the code: an optimising host
compiler may duplicate a branch around a wave operation (legal for it, since
it does not know such calls are convergent), which would look like lanes of
one wave at different operations."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_18900_amd", "csrc")
DEVICE_SOURCES = ["kernels", "noalloc", "split"]        # HIP files, compiled as host C++
HOST_SOURCES = ["runtime.cpp", "encode.cpp"]


def build(out_dir: str) -> str:
    os.makedirs(out_dir, exist_ok=True)
    srcs = []
    for name in DEVICE_SOURCES:
        dst = os.path.join(out_dir, name + ".cpp")
        shutil.copyfile(os.path.join(CSRC, name + ".hip"), dst)
        srcs.append(dst)
    srcs += [os.path.join(CSRC, s) for s in HOST_SOURCES]
    srcs += [os.path.join(HERE, "emu.cpp"), os.path.join(HERE, "emu_main.cpp")]
    exe = os.path.join(out_dir, "lz_emu")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = (["g++", "-std=c++17", "-O0", "-g", "-fno-omit-frame-pointer"] + san +
           ["-I", os.path.join(HERE, "shim"), "-I", os.path.join(ROOT, "include"), "-I", CSRC] +
           srcs + ["-o", exe, "-lpthread", "-ldl"])
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    return exe
