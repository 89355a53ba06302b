"""Host-side parts of the benchmark contract (no GPU): the single-GPU
refusal exits before touching a device, and the flop and traffic bookkeeping
the roofline figures are built from."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_assign_flops_is_two_d_k_per_point_pass():
    # one squared distance per point and center: d multiplies and d adds
    assert bench.assign_flops(n=10, d=16, k=256, assigns=3) == 2.0 * 16 * 256 * 10 * 3
    assert bench.assign_flops(n=1, d=1, k=1, assigns=0) == 0.0


def test_traffic_records_are_tied_to_the_kernel_sources():
    # a record counts only while the hash of its sources (and the build
    # script) is the one it was taken with
    h = bench.source_hash(["lloyd.hip", "lloyd_dev.h", "internal.h", "../build.py"])
    assert len(h) == 16 and h == bench.source_hash(["lloyd.hip", "lloyd_dev.h", "internal.h",
                                                    "../build.py"])
    assert h != bench.source_hash(["lloyd.hip", "lloyd_dev.h", "internal.h"])
    for cls, b in bench.measured_traffic().items():
        assert cls in ("subcluster", "lloyd_fused") and b > 0
