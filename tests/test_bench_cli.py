"""bench.py's command line, on the CPU: it measures one GPU and refuses a
larger --gpus with a message (before touching any device)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_bench_lists_workloads():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 0
    for wl in ("c1", "c2", "c3", "c4", "c5", "t1", "t2", "e2"):
        assert wl in out.stdout


def test_numpy_explicit_baseline_matches_oracle(orc):
    """The FP64 NumPy explicitly padded CPU baseline of the 3D workload
    computes the same sums as the oracle (small grid, zero-slot storage)."""
    import numpy as np
    import bench
    import synth
    m, n = (4, 5, 6), (8, 10, 7)
    f = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 300 + i) for i in range(2)])
    g = np.stack([synth.power_spectrum_centered(m, n, 11 / 6, 310 + i) for i in range(2)])
    # NO_SYMMETRIZE reading: the real transforms see the k_z = 0 plane's projection
    ref = orc.convnd_hermitian(f, g, m, symmetrize=False)
    got = bench.numpy_explicit_hermitian_3d(f, g, m, 2)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13
