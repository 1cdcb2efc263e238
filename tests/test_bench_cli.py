"""The benchmark's command line on the CPU: it measures one GPU, so more
than one is refused with a message and a non-zero status before any device
work; --help lists the legs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr


def test_help_lists_the_legs():
    r = _run("--help")
    assert r.returncode == 0
    for leg in ("tiny", "multi_pocket", "score", "local_opt", "batching", "stream_plain", "box_sweep", "surface"):
        assert leg in r.stdout
