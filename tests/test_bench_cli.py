"""The bench's command-line contract that holds without a GPU: more than
one GPU is refused with a message and exit status 2, and the help lists the
documented options."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--prec", "--workload", "--no-cpu", "--tau",
                "--max-passes", "--kerker", "--scf-runs", "--scf-only", "--max-scf-steps",
                "--profile-applies", "--prec-error"):
        assert opt in r.stdout, opt
