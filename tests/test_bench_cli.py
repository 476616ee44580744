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
