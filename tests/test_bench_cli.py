"""Command-line contract of bench.py that holds without a GPU (CPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_workloads_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("spheres191", "batch48", "cracks479", "spheres703", "walls191", "hsweep", "grad128", "hbm480"):
        assert w in r.stdout, w
