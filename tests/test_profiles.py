"""The committed rocprofv3 summaries and the bench's use of them, without a
GPU: every summary names the command that produced it (committed files only)
and the kernel sources it measured, and the bench takes a counter figure only
while that source hash matches."""

import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
sys.path.insert(0, ROOT)


def summaries():
    return sorted(f for f in os.listdir(PROFILES) if f.endswith((".txt", ".md")))


def test_every_summary_names_its_command_and_sources():
    files = summaries()
    assert files, "no profile summaries committed"
    for f in files:
        text = open(os.path.join(PROFILES, f)).read()
        assert re.search(r"^kernel_source_sha256: [0-9a-f]{64}$", text, re.M), f
        commands = re.findall(r"^command[^:]*: (.*)$", text, re.M)
        assert commands, f
        for c in commands:
            # the program after "--" is a committed file of this repository
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] == "python3" and os.path.exists(os.path.join(ROOT, prog[1])), (f, c)
        assert len(text) < 16384, f   # short summaries, not raw profiler output


def recorded_hash():
    for line in open(os.path.join(PROFILES, "hbm_traffic.txt")):
        if line.startswith("kernel_source_sha256:"):
            return line.split(":", 1)[1].strip()
    raise AssertionError("hbm_traffic.txt has no source hash")


def test_traffic_is_taken_only_for_the_measured_sources(monkeypatch):
    import bench
    monkeypatch.setattr(bench, "kernel_source_hash", recorded_hash)
    t = bench.profiled_traffic("raycast_kernel/G4", "c3-hand-1280x960/f32")
    assert t is not None and t > 0
    assert bench.profiled_traffic("fuse_kernel", "c3-hand-1280x960/f16") > 0
    assert bench.profiled_traffic("raycast_kernel/G4", "no-such-workload/f32") is None
    # other kernel sources: the counters no longer describe them
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.profiled_traffic("raycast_kernel/G4", "c3-hand-1280x960/f32") is None


def test_kernel_source_hash_covers_the_profiled_kernels():
    """Every source file the profiled kernels are built from (the launch
    files and the headers they pull in from the same folder) is hashed, so a
    change to any of them retires the committed counters."""
    import bench
    csrc = os.path.join(ROOT, "paper_1311_7194_amd", "csrc")
    todo, seen = ["fuse.hip", "raycast.hip"], set()
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        for inc in re.findall(r'^#include "([^"]+)"', open(os.path.join(csrc, f)).read(), re.M):
            if os.path.exists(os.path.join(csrc, inc)):
                todo.append(inc)
    assert seen <= set(bench.KERNEL_SOURCES), seen - set(bench.KERNEL_SOURCES)
    assert re.fullmatch(r"[0-9a-f]{64}", bench.kernel_source_hash())
