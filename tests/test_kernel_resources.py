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
       "k_step_lv", "k_yupdate", "k_lvl_jacobi0", "k_prolong_lds", "k_spmm_real_halo",
       "k_coarse_gemm", "k_pole_lists"]


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


def test_mfma_loops_keep_their_accumulators():
    """The FP64 MFMA kernels of Rayleigh-Ritz (Gram and tall GEMM: 20-25
    accumulator blocks per wave) compiled with the library's flags for their
    file: no scratch, and the loop blocks that issue the MFMAs hold no
    accumulator copies between register files (with 200 accumulator registers
    the default allocation moved every accumulator twice per MFMA round)."""
    if HIPCC is None:
        pytest.skip("hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "slrf_build", os.path.join(ROOT, "paper_2510_17334_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    out = os.path.join(os.environ.get("TMPDIR", "/tmp"), "slrf_kernels_dense_%d.s" % os.getpid())
    cmd = [HIPCC] + build.PER_FILE_FLAGS.get("kernels_dense.hip", []) + [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
        "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
        os.path.join(CSRC, "kernels_dense.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = open(out).read().splitlines()
    os.remove(out)
    starts = [(i, m.group(1)) for i, l in enumerate(lines)
              for m in [re.match(r"^(_Z\S*(k_gram|k_gemm_tall)[IE]\S*):", l)] if m]
    assert {re.search(r"(k_gram|k_gemm_tall)", f).group(1) for _, f in starts} == \
        {"k_gram", "k_gemm_tall"}
    text = "\n".join(lines)
    for st, fn in starts:
        en = next(i for i in range(st, len(lines)) if lines[i].strip().startswith(".Lfunc_end"))
        body = lines[st:en]
        cuts = [i for i, l in enumerate(body) if l.startswith(".LBB")] + [len(body)]
        mfma_blocks = 0
        for a, b in zip(cuts[:-1], cuts[1:]):
            ins = [x.strip() for x in body[a:b] if x.strip() and not x.strip().startswith((";", "."))]
            n_mfma = sum("v_mfma_f64" in x for x in ins)
            if n_mfma:
                mfma_blocks += 1
                copies = sum(x.startswith(("v_accvgpr_read", "v_accvgpr_write")) for x in ins)
                assert copies <= n_mfma // 2, (fn, n_mfma, copies)
        assert mfma_blocks > 0, fn
        m = re.search(r"\.amdhsa_kernel " + re.escape(fn) + r"\n(.*?)\.end_amdhsa_kernel", text,
                      re.S)
        assert m and int(re.search(r"\.amdhsa_private_segment_fixed_size (\d+)",
                                   m.group(1)).group(1)) == 0, fn
