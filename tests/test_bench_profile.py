"""bench.py and its committed profiles agree (no GPU needed)."""


def test_traffic_comes_only_from_a_profile_of_the_current_kernels():
    """bench.py reports the HBM traffic of k_main from the committed rocprofv3
    counter summary only while that summary was taken from the current step
    kernel sources (hash in the summary); otherwise the figure is null."""
    import json
    import os

    import bench

    path = os.path.join(os.path.dirname(bench.__file__), "profiles", "k_main_rock256_f32_pmc.md")
    meta = {}
    for line in open(path):
        if line.startswith("<!--") and "traffic:" in line:
            meta = json.loads(line.strip()[4:-3].split("traffic:", 1)[1])
    t = bench.read_traffic(meta.get("n_fluid", 0), meta.get("block", 256))
    if meta.get("kernel_hash") == bench.kernel_source_hash():
        assert t is not None and 1.0e9 < t < 1.6e9, t
    else:
        assert t is None
    assert bench.read_traffic(12345, 256) is None


def test_more_than_one_gpu_is_refused_with_a_message():
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
