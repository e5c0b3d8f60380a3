"""The benchmark's command line on the CPU: it measures one GPU and says
so, before any device work, when asked for more (there is no multi-GPU
path); its help lists the legs it runs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_help_names_the_legs():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--skip-fp32", "--skip-adjoint", "--skip-batch", "--skip-cpu", "--kernel"):
        assert flag in r.stdout, flag
