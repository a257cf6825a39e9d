"""Host checks of bench.py's command line: the one-GPU contract and the
argument parser (no GPU needed: both paths exit before any device work)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", "--steps", "1")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_workload_is_refused():
    r = _run("--workload", "C9")
    assert r.returncode != 0 and "invalid choice" in r.stderr


def test_help_lists_the_measurement_modes():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--workload", "--precision", "--kernel-sweep", "--redo-frac", "--poisson"):
        assert flag in r.stdout
