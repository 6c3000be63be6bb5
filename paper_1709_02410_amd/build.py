"""Build librpywall.so (HIP, gfx950) in-tree with hipcc.

The sources are compiled to objects in parallel (one hipcc per source, in a
temporary folder) and linked into paper_1709_02410_amd/librpywall.so.

Usage: python -m paper_1709_02410_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librpywall.so")
SOURCES = ["api.hip", "pair_kernels.hip", "krylov.hip", "lanczos.hip", "rigid.hip", "ts.hip", "vjp.hip",
           "settings.hip", "calibrate.hip", "lanczos_step.hip", "rigid_step.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed FP32 instructions out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="rpywall_build_") as tmpd:
        def compile_one(src: str):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            return obj, subprocess.run(cmd, capture_output=True, text=True)

        jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, SOURCES))
        failed = [r for _, r in results if r.returncode != 0]
        if failed:
            for r in failed:
                sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed building librpywall.so")
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in results], "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking librpywall.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
