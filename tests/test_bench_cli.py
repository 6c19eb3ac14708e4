"""bench.py's command line on the CPU: one GPU only (--gpus N > 1 exits with
a message and status 2 before any GPU work), and --help lists the flags the
benchmark's sections use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_sections():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--frac-bits", "--no-fits", "--fits-only", "--no-batch", "--no-serve",
                 "--no-lookups", "--no-queries", "--no-cpu-baseline"):
        assert flag in r.stdout, flag
