"""CPU checks of bench.py's command line: one GPU only, and the HBM-traffic
figure is reported only while the profiled kernel's source is unchanged."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_gated_by_source_hash_width_and_launch_count():
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic("gemm_c32_b3p", "default", 29)
    assert t is not None and t > 0
    assert bench.measured_traffic("gemm_c32_b3p", 256, 29) is None
    assert bench.measured_traffic("gemm_c32_b3p", "default", 30) is None
    assert len(bench.kernel_source_sha256("gemm_c32_b3p")) == 64
