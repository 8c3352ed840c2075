"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the path is built for one GPU) before anything is measured, and
--help lists the options the driver and the profiles use.  No GPU is
touched."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr + r.stdout
    assert r.stdout.strip() == ""        # no JSON line: nothing was measured


def test_help_lists_the_options():
    r = _bench("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--precision", "--no-cpu-baseline",
                "--precond"):
        assert opt in r.stdout
