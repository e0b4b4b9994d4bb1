"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU.

  * the oracle (all of oracle/*.c) built with gcc under both sanitizers and
    driven through every entry point (tests/sanitize/oracle_driver.c);
  * the host side of libtsdf (every source; the sanitizers instrument the
    host code only, and no device code runs) under both sanitizers, driven
    through its validation, sizing and table paths
    (tests/sanitize/abi_driver.cpp).
A finding aborts the driver, which fails the test.
"""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    srcs = sorted(glob.glob(os.path.join(ROOT, "oracle", "*.c")))
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")] + srcs + ["-lm"])
    out = run([exe], env=SAN_ENV, timeout=300)
    assert "triangles" in out


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="needs hipcc")
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1311_7194_amd", "csrc")]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1311_7194_amd", "csrc", "*.hip")))
    objs = []
    procs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        objs.append(o)
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
               "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
               "-Wno-unused-command-line-argument"] + inc + ["-c", s, "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    for cmd, p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"{' '.join(cmd)}\n{out}\n{err}"
    drv = str(tmp_path / "abi_driver.o")
    run([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
         "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all"] + inc +
        ["-c", os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), "-o", drv])
    # link with the compiler's own driver
    exe = str(tmp_path / "abi_driver")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    run([os.path.join(rocm, "llvm", "bin", "clang++"), "-fsanitize=address,undefined", "-o", exe, drv] + objs +
        ["-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")])
    out = run([exe], env=SAN_ENV, timeout=300)
    assert "0 failures" in out
