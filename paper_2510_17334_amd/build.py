"""Build the HIP shared library ``libslrf.so`` for gfx950, in-tree.

Usage: ``python -m paper_2510_17334_amd.build`` (or ``build()`` from Python).
Compiles every ``csrc/*.hip`` and ``csrc/*.cpp`` with hipcc into one shared
object next to this file.  Packed-FP32 instructions are disabled for all device
code (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libslrf.so")
ARCH = "gfx950"


# The MFMA kernels keep their FP64 accumulators (up to 200 registers) in the
# VGPR form: otherwise the register allocator parks them in AGPRs and copies
# them back and forth around every MFMA of the loop.
# The device AMG products round every product before adding it (no fused
# multiply-add), as the host build does, so the two hierarchies are equal.
PER_FILE_FLAGS = {"kernels_dense.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
                  "amg_device.hip": ["-ffp-contract=off"]}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = _hipcc()
    src = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                 glob.glob(os.path.join(HERE, "csrc", "*.cpp")))
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    common = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument",
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]

    def compile_one(f):
        o = os.path.join(obj_dir, os.path.basename(f) + ".o")
        cmd = [hipcc] + common + ["-c", f, "-o", o]
        if f.endswith(".cpp"):
            cmd = [hipcc] + common + ["-x", "hip", "-c", f, "-o", o]
        if os.path.basename(f) in PER_FILE_FLAGS:
            cmd[1:1] = PER_FILE_FLAGS[os.path.basename(f)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return o

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, src))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
