"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message, and an unknown workload is an error."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, cwd=ROOT, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_unknown_workload_is_an_error():
    r = _run("--workload", "nope", "--no-autotune", "--no-cpu-baseline")
    assert r.returncode == 2 and "invalid choice" in r.stderr
