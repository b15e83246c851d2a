"""Host-side behaviour of bench.py that needs no GPU: one GPU only, so --gpus above 1 exits
with a message (before anything touches a device), and the kernel source hash that keys the
committed traffic record covers the fused kernel's sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_keyed_by_the_fused_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench

    assert "paper_2602_15939_amd/csrc/gpd.hip" in bench.GPD_SOURCES
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
