"""bench.py and its committed profiles agree (no GPU needed)."""


def test_committed_traffic_profile_matches_the_step_kernel_sources():
    """bench.py reports the HBM traffic of k_main from the committed rocprofv3
    counter summary only while that summary was taken from the current step
    kernel sources; this keeps the two in step (a kernel change needs a new
    profile)."""
    import bench

    t = bench.read_traffic(4624221, 256)
    assert t is not None and 1.2e9 < t < 1.6e9, t


def test_more_than_one_gpu_is_refused_with_a_message():
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
