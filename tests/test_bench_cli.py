"""The benchmark's command line on the CPU: it measures one GPU, so more
than one is refused with a message and a non-zero status before any device
work; --help lists the legs; the recorded HBM traffic is used only where it
still describes the code."""
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


def test_recorded_traffic_only_for_matching_sources_and_order():
    """The HBM traffic in the bench line comes from the committed counter
    record only while every native source hashes to the recorded value and
    the job order is the recorded one; otherwise it is null."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    rec = None
    for line in open(os.path.join(ROOT, "profiles", "dock_kernel_screening_stream.md")):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
    assert rec is not None and rec["job_order"] in ("stream", "box")
    other = "stream" if rec["job_order"] == "box" else "box"
    assert bench.recorded_traffic(other) is None
    got = bench.recorded_traffic(rec["job_order"])
    if bench.native_source_hash() == rec["native_source_sha256"]:
        assert got == rec["dock_traffic_bytes_per_launch"]
    else:
        assert got is None


def test_flop_counts():
    """The roofline's count is F = 70 P + 90 N + 60 T per evaluation, every
    evaluation in full; the work performed takes out 70 P for each trial the
    intra bound decides, and nothing else."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    assert bench.flops_of(3, 100, 20, 5) == 3 * (70 * 100 + 90 * 20 + 60 * 5)
    ev, bnd = np.array([10, 7, 0]), np.array([4, 0, 0])
    P, N, T = np.array([100, 50, 10]), np.array([20, 12, 8]), np.array([5, 0, 1])
    full = bench.flops_of(ev, P, N, T)
    done = bench.flops_performed(ev, bnd, P, N, T)
    assert np.array_equal(full - done, bnd * 70 * P)
    assert np.array_equal(bench.flops_performed(ev, 0, P, N, T), full)
