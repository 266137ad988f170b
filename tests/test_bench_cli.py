"""bench.py's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_and_byte_models():
    import bench
    work = {"flops_rhs": 1000.0, "flops_jac": 5000.0}
    na = np.array([2, 1])
    nr = np.array([1, 0])
    n = 10
    f_lu = n * (n - 1) / 2 + (n - 1) * n * (2 * n - 1) / 3
    f_att = 2 * 1000.0 + (n + 1) + f_lu + 4 * (2 * n * n - n) + 35 * n
    assert bench.flops_per_launch(work, n, na, nr) == 3 * 6000.0 + 4 * f_att
    b = bench.bytes_per_launch_wide(161, na, nr, 2)
    assert b == 64.0 * 161 * 161 * 4 + 24.0 * 161 * 161 * 3 + 2 * 8 * 162 * 2


def test_counters_only_for_the_profiled_sources():
    import hashlib
    import bench
    t = bench.measured_traffic()
    assert t is None or t > 2.3e8          # at least phi in and out of 262144 cells
    e = bench.measured_fp64_ops()
    assert e is None or e > 1e12
    srcs = bench.WAVE_KERNEL_SOURCES
    cur = {s: hashlib.sha256(open(os.path.join(ROOT, "paper_2112_05834_amd", "csrc", s), "rb")
                             .read()).hexdigest()[:16] for s in srcs}
    text = "; ".join("%s sha256 prefix %s" % (s, cur[s]) for s in srcs)
    assert bench._sources_current(text, srcs)
    # a stale prefix for either source, or a missing one, makes the figures unusable
    for s in srcs:
        stale = text.replace(cur[s], "0" * 16)
        assert not bench._sources_current(stale, srcs)
    assert not bench._sources_current(text.split("; ")[0], srcs)
