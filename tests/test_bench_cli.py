"""The bench's command-line contract that needs no GPU: more than one GPU is
refused with a message (the build measures one GPU; sharding is a design
note), and the help text lists the legs' switches."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_legs():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-serve", "--serve-requests", "--precision",
                 "--profile-target"):
        assert flag in r.stdout
