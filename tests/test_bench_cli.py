"""CPU checks of bench.py's command line: one GPU only, and the HBM-traffic
figure is reported only while the profiled kernel's source, the block width
and the mix of launch sizes (the algorithmic bytes per launch) are those the
counters were taken with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_gated_by_source_hash_width_and_launch_mix(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_source_sha256("gemm_3m")
    assert len(sha) == 64
    (tmp_path / "pmc_gemm_3m_two_spheres_N5124_nk512.txt").write_text(
        f"kernel_source_sha256: {sha}\nblock_width: default\nalgorithmic_bytes_per_launch: 3.909e9\n"
        "traffic_bytes_per_launch: 1.5e9\n")
    d = str(tmp_path)
    assert bench.measured_traffic("gemm_3m", "default", 3.9093e9, profiles=d) == 1.5e9
    assert bench.measured_traffic("gemm_3m", 256, 3.909e9, profiles=d) is None
    assert bench.measured_traffic("gemm_3m", "default", 3.92e9, profiles=d) is None
    assert bench.measured_traffic("gemm_c32", "default", 3.909e9, profiles=d) is None
    (tmp_path / "pmc_gemm_3m_two_spheres_N5124_nk512.txt").write_text(
        "kernel_source_sha256: 00\nblock_width: default\nalgorithmic_bytes_per_launch: 3.909e9\n"
        "traffic_bytes_per_launch: 1.5e9\n")
    assert bench.measured_traffic("gemm_3m", "default", 3.909e9, profiles=d) is None
    # the committed summary applies to the default sweep's mix
    assert bench.measured_traffic("gemm_3m", "default", 3.909040e9) is not None
