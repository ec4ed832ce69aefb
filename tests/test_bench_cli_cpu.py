"""The benchmark's command line on the CPU: more than one GPU is refused with a
message before anything touches a GPU (the engine and its measurements use one
GPU; sharding over several is a design only)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert p.returncode == 2, (n, p.returncode, p.stderr[-500:])
        assert "one GPU only" in p.stderr
        assert p.stdout == ""  # no JSON line: nothing was measured
