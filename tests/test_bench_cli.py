"""bench.py's command line on the host: more than one GPU is refused with a
message (the path runs on one GPU), and the counter records are read only
when they were taken on the current step kernels."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_records_follow_the_kernel_sources(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    good = tmp_path / "traffic.txt"
    good.write_text(f"kernel_source_hash = {h}\nhbm_bytes_per_launch = 123456\n")
    assert bench.measured_traffic(str(good)) == 123456.0
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_hash = 0000000000000000\nhbm_bytes_per_launch = 1\n")
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None
