"""bench.py's contract on the CPU: a multi-GPU request is refused with a message
(this build measures one GPU), and the committed counter summary of the sweep
was taken on the sources that are built, so the bench line reports its HBM
traffic instead of null."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiled_sweep_traffic_matches_the_sources():
    import bench
    t = bench.profiled_traffic()
    assert t is not None, "profiles/ summary taken on other sweep sources"
    # the c64 sweep moves several GB per launch at the benchmark workload
    assert 1e9 < t < 1e11
