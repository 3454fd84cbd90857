"""Host-side checks of bench.py's command line (no GPU is touched)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    for extra in ([], ["--workload", "vjp"]):
        r = _bench("--gpus", "2", *extra)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""
