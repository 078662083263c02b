"""The decode kernel's occupancy contract, checked on the compiled gfx950 code
(no GPU needed): three workgroups of 256 threads per CU, i.e. three waves per
SIMD, needs at most 168 VGPRs, no scratch (spilled registers) and at most a
third of the CU's 160 KiB of LDS per workgroup."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def kernel_meta(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    from paper_2606_18900_amd.build import FLAGS
    flags = [f for f in FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [HIPCC] + flags + ["-x", "hip", "--cuda-device-only", "-S",
                             os.path.join(ROOT, "paper_2606_18900_amd", "csrc", "kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    text = out.read_text()
    # the kernel descriptor of k_decode
    m = re.search(r"\.amdhsa_kernel \S*k_decode\S*\n(.*?)\.end_amdhsa_kernel", text, re.S)
    assert m, "k_decode descriptor not found"
    desc = m.group(1)
    get = lambda key: int(re.search(r"\." + key + r" (\d+)", desc).group(1))
    return {"vgpr": get("amdhsa_next_free_vgpr"), "scratch": get("amdhsa_private_segment_fixed_size"),
            "lds": get("amdhsa_group_segment_fixed_size")}


def test_three_waves_per_simd(kernel_meta):
    assert kernel_meta["vgpr"] <= 168, kernel_meta
    assert kernel_meta["scratch"] == 0, kernel_meta


def test_three_workgroups_per_cu_lds(kernel_meta):
    assert 3 * kernel_meta["lds"] <= 160 * 1024, kernel_meta
