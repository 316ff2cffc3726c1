"""Register budget of the hot kernels (no GPU needed): the device code of
kernels_block.hip, compiled for gfx950 with the library's flags, keeps every
hot kernel free of scratch (private) memory.  A per-thread array that the
compiler fails to keep in registers (the halo prefetch of the tile kernels is
one) lands in scratch and slows its kernel severalfold without changing any
result, so no numeric test would notice."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_17334_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")

# kernels of the filter's inner loop (mangled-name fragments)
HOT = ["k_apply_halo", "k_true_halo", "k_post_image", "k_restrict", "k_orth_lv", "k_dots_lv",
       "k_step_lv", "k_yupdate", "k_lvl_jacobi0", "k_prolong_lds", "k_coarse_solve"]


@pytest.fixture(scope="module")
def descriptors(tmp_path_factory):
    if HIPCC is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "kernels_block.s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "kernels_block.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    text = open(out).read()
    found = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)\n(.*?)\.end_amdhsa_kernel", text, re.S):
        body = m.group(2)
        scratch = int(re.search(r"\.amdhsa_private_segment_fixed_size (\d+)", body).group(1))
        vgpr = int(re.search(r"\.amdhsa_next_free_vgpr (\d+)", body).group(1))
        found[m.group(1)] = (scratch, vgpr)
    return found


def test_hot_kernels_use_no_scratch(descriptors):
    hot = {k: v for k, v in descriptors.items() if any(h in k for h in HOT)}
    # every family is present (a rename would otherwise empty the check)
    for h in HOT:
        assert any(h in k for k in hot), h
    spilled = {k: v for k, v in hot.items() if v[0] != 0}
    assert not spilled, spilled
    # and within the 512 registers a lane can address
    assert max(v[1] for v in hot.values()) <= 512
