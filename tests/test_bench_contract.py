"""Host-side checks of the benchmark's command-line contract (no GPU needed): more than one GPU is
refused with a message and a non-zero exit before anything touches a device, and the workload
generator matches the documented configuration."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                           env={**os.environ, **env}, timeout=120)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_workload_shape():
    sys.path.insert(0, ROOT)
    import bench
    wl = bench.setup_workload(n=64, m=5000, R=8)
    assert wl["uv"].shape == (5000, 2) and wl["uv"].dtype == np.float64
    assert np.all(np.abs(wl["uv"]) <= np.pi)
    assert len(wl["off"]) == 9 and wl["off"][0] == 0 and wl["off"][-1] == 5000
    assert np.all(np.diff(wl["off"]) > 0)
    assert wl["x_true"].shape == (64, 64) and wl["x_true"].max() == np.float32(1.0)
    r = np.hypot(wl["uv"][:, 0], wl["uv"][:, 1])
    assert np.all(np.diff(r) >= 0)   # sorted by radius: the blocks are annuli
