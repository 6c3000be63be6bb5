"""AddressSanitizer + UndefinedBehaviorSanitizer builds (host code, g++) of
the FP64 oracle and of the device pair arithmetic compiled for the CPU, each
driven by a small program that calls every entry point on inputs with
blobs below the wall, overlapping and coincident pairs and cross-checks the
results.  Any memory error or undefined behaviour aborts the program."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, name, sources, extra=()):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", *SAN, *extra, *sources, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, "san_oracle",
                   [os.path.join(ROOT, "oracle", "rpy_oracle.cpp"), os.path.join(HARNESS, "sanitize_oracle_main.cpp")],
                   extra=["-fopenmp", "-ffp-contract=off"])


def test_pair_math_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, "san_pair_math",
                   ["-I", HARNESS, os.path.join(HARNESS, "pair_math_host.cpp"),
                    os.path.join(HARNESS, "sanitize_pair_math_main.cpp")], extra=["-ffp-contract=off"])
