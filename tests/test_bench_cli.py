"""bench.py's command line: more than one GPU is refused with a message (the
path shards by particles, but one GPU is what is measured), and the help lists
the workload, tolerance, precision, cache and timing options.  Both exit
before touching a device, so they are safe on any machine."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_workload_and_tolerance_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--workload", "--tol", "--precision", "--cache-cells", "--steps", "--warmup"):
        assert opt in r.stdout, opt
