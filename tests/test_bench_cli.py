"""bench.py's command-line contract, on the CPU: a request for more than one
GPU exits with a message (this build measures one GPU), and --help lists every
measurement mode."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_every_mode():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--exact-scaling", "--em3d", "--variants",
                 "--precision-form", "--apply-burst", "--mix", "--batch-cols",
                 "--copy-calibration", "--no-cpu-baseline", "--compose",
                 "--solve-rounds"):
        assert flag in r.stdout, flag
