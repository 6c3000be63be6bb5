"""The algorithmic FLOP constants the benchmark reports against the vector
peak are the counts of the device pair arithmetic itself: pair_math.h is
compiled for the CPU with a counting scalar type (FMA = 2, add/sub/mul = 1,
rsqrt = 1; terms of the target blob alone are not counted per pair) and the
counts must equal bench.py's constants.  Runs without a GPU."""
import importlib.util
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_consts", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_flop_constants_match_the_counted_formula(tmp_path):
    exe = str(tmp_path / "flop_count")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HARNESS, os.path.join(HARNESS, "flop_count.cpp"), "-o", exe],
                   check=True)
    counts = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    b = _bench()
    assert counts == {"shared": b.FLOP_PAIR_SHARED, "apply": b.FLOP_PAIR_RHS, "block": b.FLOP_PAIR_BLOCK,
                      "block_apply": b.FLOP_BLOCK_RHS, "vjp_pair": b.FLOP_VJP_PAIR, "vjp_self": b.FLOP_VJP_SELF}
    # symmetric product of N blobs: N(N-1)/2 unordered pairs (geometry once,
    # two applications) plus N self pairs (one application)
    N = 10
    assert b.algorithmic_flop(N, 1, 1) == 45 * (counts["shared"] + 2 * counts["apply"]) + 10 * (
        counts["shared"] + counts["apply"])
    assert b.algorithmic_flop(N, 2, 0) == 100 * (counts["shared"] + 2 * counts["apply"])
    assert b.vjp_flop(N, 1) == 45 * counts["vjp_pair"] + 10 * counts["vjp_self"]
    # matrix-core multi-RHS kernel: every ordered pair forms its block once
    # (vector units) and contracts it with each right-hand side (matrix cores)
    assert b.mat_flop(N, 16) == (100 * (counts["shared"] + counts["block"]), 100 * 16 * counts["block_apply"])
