"""The benchmark's command line on a machine without a GPU: more than one GPU is refused
with a message before any device work, and the state-based profiling mode insists on the
staged FP64/FP32 configuration it times."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_state_based_mode_needs_the_staged_mapping():
    r = _run("--model", "state_based", "--mapping", "sliced", "--no-extras", "--no-cpu-baseline")
    assert r.returncode != 0 and "staged" in r.stderr
