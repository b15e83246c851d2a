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


def test_algorithmic_bytes_follow_the_method_not_the_implementation():
    """56 B per particle (16 B position + 12 B momentum, read and written) and 48 B per cell for
    the 3D boxes; the sort permutation read is implementation traffic, reported apart."""
    sys.path.insert(0, ROOT)
    import bench

    w = bench.workload_shear3d(n=256)
    n = 268_435_456
    assert bench.algorithmic_bytes(w, n) == n * 56 + 256**3 * 48  # 1.584e10 B
    assert bench.implementation_bytes(w, n) == n * 4
    from paper_2602_15939_amd import workloads

    leaky = workloads.WORKLOADS["leaky2d"]()
    assert bench.algorithmic_bytes(leaky, 1) == 48 + 4 + 2048**2 * 48
    paper = workloads.WORKLOADS["leaky2d_paper"]()
    assert bench.algorithmic_bytes(paper, 1) == 48 + 4 + 16 + 2048**2 * 48


def test_cpu_model_is_named():
    sys.path.insert(0, ROOT)
    import bench

    assert bench.cpu_model() and bench.cpu_model() != "unknown"
