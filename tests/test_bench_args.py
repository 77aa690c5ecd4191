"""bench.py refuses what it does not run before it touches the GPU: more than
one GPU (the multi-GPU layout is a design note) and the corner push followed
by the dual push on the batch workload (a single-LP option)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_both_pushes_on_the_batch_are_refused():
    r = _run("--config", "c3", "--push", "both")
    assert r.returncode == 2
    assert "single-LP" in r.stderr
