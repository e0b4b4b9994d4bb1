"""Command-line contract of bench.py that holds without a GPU: more than
one GPU is refused with a message, and a host without a visible GPU gets an
error instead of a CPU fallback."""

import json
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    return r.returncode, r.stdout.strip().splitlines()


def test_more_than_one_gpu_is_refused():
    rc, out = run_bench("--gpus", "2")
    assert rc == 2
    assert "one GPU only" in json.loads(out[-1])["error"]


@pytest.mark.skipif(torch.cuda.is_available(), reason="needs a host without a GPU")
def test_no_gpu_is_an_error_not_a_fallback():
    rc, out = run_bench("--steps", "1", "--warmup", "0")
    assert rc == 1
    assert json.loads(out[-1]) == {"error": "no GPU visible"}


def test_raycast_group_takes_only_the_built_group_sizes():
    # the raycast kernels are instantiated for 1, 2, 4, 8 and 16 lanes per ray
    rc, _ = run_bench("--raycast-group", "3")
    assert rc == 2
    rc, _ = run_bench("--gpus", "2", "--raycast-group", "8")
    assert rc == 2   # parsed, then refused for the GPU count
