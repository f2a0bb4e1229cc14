"""Host-side checks of bench.py's contract that need no GPU: more than one GPU
is refused with a message before anything touches a device, and the stored
HBM counter record matches the simulation kernel's current sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                           env=dict(os.environ, **env), timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_traffic_record_matches_the_kernel_sources():
    """The counter record is keyed on a hash of the kernel's sources; a change
    to them without new counters makes the bench report null traffic."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    assert t is not None and 1e5 < t < 1e8


def test_config3_sides_are_uniform_over_all_seven():
    """The uneven workload draws every side 64, 96, .., 256 (lattices 64 x 64
    to 256 x 256, uniform per protocol) and whole-day horizons of 10-40 days."""
    import numpy as np
    from paper_2303_08123_amd import workloads
    lattice, horizon = workloads.config3_shapes(8192, seed=0)
    counts = np.bincount(lattice // 32 - 2, minlength=7)
    assert set(np.unique(lattice).tolist()) == {64, 96, 128, 160, 192, 224, 256}
    assert counts.min() > 8192 / 7 * 0.85
    assert horizon.min() >= 240 and horizon.max() <= 960 and np.all(horizon % 24 == 0)
