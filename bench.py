#!/usr/bin/env python3
"""Benchmark of the wall-corrected RPY blob mobility on one MI355X.

Metric: blob-pair interactions per second of the dense product u = M(r) f
(FP32 pair terms with compensated sums, and FP64), on 1e5 free blobs with
the config-0 density (x, y ~ U[0, 600], z ~ U[1.1, 6], a = eta = 1,
f ~ N(0,1), seed 0).  A timed step is one product: pack (O(N)), the O(N^2)
pair kernel and the epilogue, inputs resident in HBM.  The same run also
times the other parts of the hot path on their own workloads (FP64 product,
16-RHS product, batched suspensions against per-instance launches,
preconditioned Lanczos, VJP, divergence) and the FP64 CPU oracle on a
bounded sample of the headline product.

Every result carries its error against the FP64 CPU oracle (relative L2
and largest entry error over the largest reference entry, on all rows or on
sampled rows), computed after the timed GPU work in the oracle leg of this
script, which also times the oracle itself (the CPU baseline).

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "wall-RPY blob-pair interactions/s (FP32 vs FP64) at 1e5 blobs; % vector peak"
PEAK_FP32 = 157.3  # TFLOP/s, MI355X FP32 vector
PEAK_FP64 = 78.6   # TFLOP/s, MI355X FP64 vector
# Algorithmic FLOPs of the pair formula (FMA = 2, add/sub/mul = 1, rsqrt = 1,
# negation/compare/select = 0; target-only terms and the FP32 precision
# bookkeeping not counted), as counted by tests/host_harness/flop_count.cpp
# on the device arithmetic itself (a test keeps these equal to its output):
# geometry and coefficients of one pair, one application M_ij f_j, one
# unordered pair of the symmetric VJP (gradient, both blobs' sums, four
# products) and one pair seen from its target only.
FLOP_PAIR_SHARED = 75
FLOP_PAIR_RHS = 24
FLOP_VJP_PAIR = 460
FLOP_VJP_SELF = 406
# The matrix-core multi-RHS kernel: the 3 x 3 block written out from the
# coefficients (vector units), and its contraction with one right-hand side
# (matrix cores), counted the same way.
FLOP_PAIR_BLOCK = 19
FLOP_BLOCK_RHS = 18
PEAK_FP32_MATRIX = 157.3  # TFLOP/s, MI355X dense FP32 matrix cores
PEAK_FP64_MATRIX = 78.6   # TFLOP/s, MI355X dense FP64 matrix cores
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernel_traffic.json")
# sources of the single-RHS pair kernels whose stored counter figures the hash
# guards (the matrix-core multi-RHS kernels of mat_pairs.h are not among them)
KERNEL_SOURCES = ["pair_kernels.hip", "pair_math.h", "records.h", "sym_pairs.h"]


def algorithmic_flop(N: int, k: int, sym: int) -> float:
    """Algorithmic FLOPs of one product of N blobs and k RHS.  The plain
    kernel evaluates every ordered pair (75 + 24 k each); the symmetric
    kernel evaluates each unordered pair once and applies it both ways
    (75 + 48 k), self pairs once (75 + 24 k)."""
    n = float(N)
    if sym:
        return n * (n - 1) / 2 * (FLOP_PAIR_SHARED + 2 * k * FLOP_PAIR_RHS) + n * (FLOP_PAIR_SHARED + k * FLOP_PAIR_RHS)
    return n * n * (FLOP_PAIR_SHARED + k * FLOP_PAIR_RHS)


def mat_flop(N: int, k: int):
    """(vector-unit, matrix-core) algorithmic FLOPs of one product of N blobs
    and k RHS on the matrix-core kernel: every ordered pair forms its block
    once (75 + 19) and contracts it with each right-hand side (18 each)."""
    n = float(N)
    return n * n * (FLOP_PAIR_SHARED + FLOP_PAIR_BLOCK), n * n * k * FLOP_BLOCK_RHS


def vjp_flop(N: int, sym: int) -> float:
    """Algorithmic FLOPs of one VJP launch: the symmetric kernel evaluates each
    unordered pair once for both blobs, self pairs from the target only; the
    plain kernel every ordered pair from its target."""
    n = float(N)
    return n * (n - 1) / 2 * FLOP_VJP_PAIR + n * FLOP_VJP_SELF if sym else n * n * FLOP_VJP_SELF


def kernel_hash() -> str:
    """Hash of the pair-kernel sources with comments and blank space removed
    (so that edits to comments alone keep the stored counter figures)."""
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1709_02410_amd", "csrc", s)) as fh:
            text = fh.read()
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()[:16]


def stored_traffic(shape: dict):
    """HBM bytes per launch of the headline pair kernel from the committed
    counter runs, or None when the kernel sources changed since or the
    counters were taken with another launch shape than `shape`."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    keys = ("sym", "ipw") if shape.get("sym") else ("sym", "tpl", "tile")
    for e in t.get("shapes", []):
        if all(e["shape"].get(k) == shape.get(k) for k in keys):
            return e["bytes_per_launch"]
    return None


def sample_rows(N: int, n: int, seed: int):
    """n distinct target rows: the first, the last (ragged tail) and n - 2
    drawn at random."""
    import numpy as np
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, N - 1), min(n - 2, max(N - 2, 0)), replace=False) if N > 2 else []
    return np.unique(np.concatenate([[0, N - 1], mid]).astype(np.int64))


def errors(got, ref) -> dict:
    """Relative L2 error and largest entry error over the largest reference
    entry of got against the oracle's ref."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    return {"rel_l2_vs_oracle": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "max_entry_vs_oracle": float(np.abs(d).max() / np.abs(ref).max())}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class _ProgressRows(dict):
    """The benchmark's rows; each one prints a progress line on stderr as it
    is filled, so a long run shows where it is."""

    def __setitem__(self, key, value):
        super().__setitem__(key, value)
        print(f"[bench] row {key} done", file=sys.stderr, flush=True)


def oracle_leg(checks, H, args, out_rows, top):
    """The CPU leg of the benchmark: the FP64 oracle (test infrastructure,
    never on the product path) evaluates every queued check on the host and
    the errors are attached to the rows; then the oracle's own throughput is
    timed on a bounded sample of the headline product, on all host cores and
    on one core."""
    import numpy as np

    from oracle import oracle as orc
    from paper_1709_02410_amd import workloads as wl
    orc.build()
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nthreads = max(1, min(nthreads, os.cpu_count() or 1))
    t_checks = time.perf_counter()
    cache = {}
    for c in checks:
        kind = c["kind"]
        try:
            if kind == "matvec":
                ref = orc.matvec(c["pos"], c["f"], rows=c.get("rows"), nthreads=nthreads, box=c.get("box"))
                e = errors(c["got"], ref)
            elif kind == "vjp":
                gp, gf = orc.vjp(c["pos"], c["f"], c["g"], rows=c["rows"], nthreads=nthreads)
                ep, ef = errors(c["got"][0], gp), errors(c["got"][1], gf)
                e = {"grad_pos": ep, "grad_f": ef,
                     "rel_l2_vs_oracle": max(ep["rel_l2_vs_oracle"], ef["rel_l2_vs_oracle"]),
                     "max_entry_vs_oracle": max(ep["max_entry_vs_oracle"], ef["max_entry_vs_oracle"])}
            elif kind == "lanczos":
                key = ("lanczos", c["name"], c["tol"])
                if key not in cache:
                    cache[key] = orc.lanczos_sqrt(c["pos"], c["W"], c["offs"], tol=c["tol"])
                ref, it_o, _, ok_o = cache[key]
                e = errors(c["got"], ref)
                e.update({"oracle_iterations": it_o, "oracle": f"oracle Lanczos at the same tolerance {c['tol']:g}"})
            elif kind == "rigid":
                key = ("rigid", c["name"], c["tol"])
                if key not in cache:
                    cache[key] = orc.rigid_gmres(c["pos"], c["q"], c["offs"], None, c["FT"], tol=c["tol"],
                                                 max_iter=200, nthreads=nthreads, box=c.get("box"))
                _, U_o, it_o, _, ok_o = cache[key]
                e = errors(c["got"], U_o)
                e.update({"oracle_iterations": it_o, "oracle": f"oracle GMRES at the same tolerance {c['tol']:g}"})
            elif kind == "divergence":
                e = errors(c["got"], orc.divergence(c["pos"], nthreads=nthreads))
            else:
                raise ValueError(kind)
        except MemoryError:
            e = {"rel_l2_vs_oracle": None, "note": "oracle out of memory"}
        e["compared"] = c["what"]
        print(f"[bench] oracle check {c['row'] or c['key']} done", file=sys.stderr, flush=True)
        if c["row"] is None:
            top[c["key"]] = e
        else:
            out_rows[c["row"]][c.get("key", "error_vs_oracle")] = e
    t_checks = time.perf_counter() - t_checks

    # oracle throughput on the headline product: all cores, then one core
    fh = wl.gaussian(H.pos.shape, 1)
    N = H.N
    rng = np.random.default_rng(0)

    def rate(threads, seconds):
        probe = rng.choice(N, 2 * threads, replace=False)
        t0 = time.perf_counter()
        orc.matvec(H.pos, fh, rows=probe, nthreads=threads)
        r = len(probe) * N / (time.perf_counter() - t0)
        nrows = int(min(N, max(len(probe), seconds * r / N)))
        rows_s = rng.choice(N, nrows, replace=False)
        t0 = time.perf_counter()
        orc.matvec(H.pos, fh, rows=rows_s, nthreads=threads)
        dt = time.perf_counter() - t0
        return nrows * N / dt, nrows, dt

    v_all, n_all, dt_all = rate(nthreads, args.cpu_seconds)
    v_one, n_one, dt_one = rate(1, args.cpu_seconds / 2)
    return {"value": v_all, "unit": "pair interactions/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n_all} random target rows x all {N} sources of the headline product, FP64, {dt_all:.1f} s "
                      f"(C++ double loop, OpenMP); rate scales linearly to the full product (rows are independent)",
            "value_1core": v_one,
            "sample_1core": f"{n_one} random target rows x all {N} sources, one thread, {dt_one:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "oracle_checks_s": round(t_checks, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--headline-only", action="store_true", help="time only the headline product")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--calib-valu", action="store_true",
                    help="also run the library's calibration kernels of known FMA count (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (the CPU baseline and every error against the oracle)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--only", action="append", default=[],
                    help="time only the extra rows whose names contain this text (repeatable; the headline "
                         "and the FP64 product always run)")
    ap.add_argument("--force-ipw", type=int, default=0,
                    help="after tuning, force the symmetric headline kernel with this many items per workgroup "
                         "(for counter runs of one launch shape)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(how the product would shard by target rows is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1709_02410_amd import rpywall as rp
    from paper_1709_02410_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    rp.lib()

    def T(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    def H2(x):
        return x.detach().cpu().numpy()

    def sync():
        torch.cuda.synchronize()

    def timed(fn, steps, warmup):
        """Wall time per call over `steps` calls, then the library-recorded
        pair-kernel time (HIP events on the launch stream) from as many calls
        again; the events add work to the stream, so the wall-clock loop
        runs without them."""
        for _ in range(warmup):
            fn()
        sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        sync()
        wall = (time.perf_counter() - t0) / steps
        rp.profile_enable(True)
        rp.profile_read(True)
        for _ in range(steps):
            fn()
        sync()
        kms, launches, pairs = rp.profile_read(True)
        rp.profile_enable(False)
        return wall, kms, launches, pairs

    def want(*names):
        """Whether any of these rows is selected (all are without --only)."""
        return not args.only or any(o in n for o in args.only for n in names)

    checks = []  # evaluated by the oracle leg after all GPU work

    def check_matvec(row, what, pos_np, f_np, got_rows, rows=None, box=None, key="error_vs_oracle"):
        checks.append({"kind": "matvec", "row": row, "key": key, "what": what, "pos": pos_np, "f": f_np,
                       "rows": rows, "got": got_rows, "box": box})

    out = {}
    rows_out = _ProgressRows()
    # ---------------------------------------------------------- headline
    H = wl.headline(seed=0)
    N = H.N
    pos = T(H.pos)
    f_np = wl.gaussian(H.pos.shape, 1)
    f = T(f_np)
    vel = torch.empty_like(f)
    F1 = f.view(1, N, 3)
    rp.autotune(pos, F1, precision=rp.FP32C)
    rp.autotune(pos, F1, precision=rp.FP64)
    if args.force_ipw:
        rp.set_shape(rp.FP32C, N, 1, tpl=1, tile=256, kblk=1, sym=1, ipw=args.force_ipw)
    step = lambda: rp.matvec(pos, f, precision=rp.FP32C, out=vel)  # noqa: E731
    wall, kms, launches, pairs = timed(step, args.steps, args.warmup)
    kavg = kms / launches
    value = N * N / wall
    shape32 = rp.get_shape(rp.FP32C, N, 1)
    flop_launch = algorithmic_flop(N, 1, shape32["sym"])
    achieved = flop_launch / (kavg * 1e-3) / 1e12
    traffic = stored_traffic(shape32)
    kname = ("sym_kernel<float, ProductBody<float,1,0>, 4> (each unordered pair once, both directions)"
             if shape32["sym"] else f"pair_kernel<float,1,{shape32['tpl']},{shape32['tile']}>")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32, 4), "traffic": traffic,
                "kernel": kname + ", FP32 pair terms, compensated sums", "shape": shape32,
                "kernel_ms_avg": round(kavg, 4), "flop_per_launch": flop_launch,
                "flop_count": {"per_unordered_pair": FLOP_PAIR_SHARED + 2 * FLOP_PAIR_RHS,
                               "per_self_pair": FLOP_PAIR_SHARED + FLOP_PAIR_RHS,
                               "shared_geometry": FLOP_PAIR_SHARED, "per_application": FLOP_PAIR_RHS,
                               "rule": "FMA 2, add/sub/mul 1, rsqrt 1; target-only terms and FP32 bookkeeping "
                                       "not counted"}}
    hrows = sample_rows(N, 256, 11)
    check_matvec(None, f"256 sampled rows of {N}", H.pos, f_np, H2(vel)[hrows], hrows, key="headline")

    if args.calib_valu:
        # 2048 blocks x 4 waves; FP32: 8 x 20000 FMA instructions per wave,
        # FP64: 8 x 5000
        calib = {}
        for kind, iters, name in ((0, 20000, "fp32"), (1, 5000, "fp64")):
            rp.calibrate(kind, 2048, iters)
            sync()
            waves = 2048 * 4
            calib[name] = {"kernel": "calib_fma_kernel<" + ("float" if kind == 0 else "double") + ">",
                           "fma_instructions": waves * 8 * iters, "flop": waves * 8 * iters * 64 * 2}
        out["calib_valu"] = calib

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        out["calib_copy_bytes"] = src.numel() * 8

    # FP64 product on the same input
    vel64 = torch.empty_like(f)
    step64 = lambda: rp.matvec(pos, f, precision=rp.FP64, out=vel64)  # noqa: E731
    w64, k64, l64, p64 = timed(step64, max(3, args.steps // 2), 1)
    shape64 = rp.get_shape(rp.FP64, N, 1)
    a64 = algorithmic_flop(N, 1, shape64["sym"]) / (k64 / l64 * 1e-3) / 1e12
    out["fp64"] = {"value": N * N / w64, "unit": "pair interactions/s", "ms_per_step": w64 * 1e3,
                   "kernel_ms_avg": k64 / l64, "shape": shape64,
                   "roofline": {"bound": "alu", "achieved": round(a64, 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
                                "frac": round(a64 / PEAK_FP64, 4)}}
    check_matvec(None, f"256 sampled rows of {N}", H.pos, f_np, H2(vel64)[hrows], hrows, key="fp64_headline")
    del vel64

    rows = rows_out
    if not args.headline_only:
        # 16-RHS product on the headline geometry
        if want("multi_rhs"):
            k = 16
            F16_np = wl.gaussian((k, N, 3), 2)
            F16 = T(F16_np)
            U16 = torch.empty_like(F16)
            rp.autotune(pos, F16, precision=rp.FP32C)
            w, km, ln, pr = timed(lambda: rp.matvec_multi(pos, F16, precision=rp.FP32C, out=U16), 3, 1)
            sh16 = rp.get_shape(rp.FP32C, N, k)
            call_ms = km / 3  # kernel time of one call (three timed calls)
            row = {"pair_rhs_per_s": k * N * N / w, "ms": w * 1e3, "kernel_ms": call_ms, "shape": sh16}
            if sh16["mat"]:
                fv, fm = mat_flop(N, k)
                tv, tm = fv / (call_ms * 1e-3) / 1e12, fm / (call_ms * 1e-3) / 1e12
                row.update({"tflops_alg": tv + tm, "bound": "mfma",
                            "matrix_tflops": tm, "frac_fp32_matrix_peak": tm / PEAK_FP32_MATRIX,
                            "vector_tflops": tv, "frac_fp32_vector_peak": tv / PEAK_FP32})
                # the same product with the contraction on the vector units
                rp.set_shape(rp.FP32C, N, k, tpl=1, tile=256, kblk=16, sym=0, ipw=4, mat=0)
                wv, kmv, _, _ = timed(lambda: rp.matvec_multi(pos, F16, precision=rp.FP32C, out=U16), 2, 1)
                rp.reset_shape(rp.FP32C, N, k)
                fl = algorithmic_flop(N, k, 0)
                row["vector_kernel"] = {"ms": wv * 1e3, "kernel_ms": kmv / 2,
                                        "tflops_alg": fl / (kmv / 2 * 1e-3) / 1e12,
                                        "frac_fp32_peak": fl / (kmv / 2 * 1e-3) / 1e12 / PEAK_FP32}
                rp.matvec_multi(pos, F16, precision=rp.FP32C, out=U16)
            else:
                fl = sum(algorithmic_flop(N, min(sh16["kblk"], k - k0), sh16["sym"])
                         for k0 in range(0, k, sh16["kblk"]))
                row.update({"tflops_alg": fl / (call_ms * 1e-3) / 1e12, "bound": "alu",
                            "frac_fp32_peak": fl / (call_ms * 1e-3) / 1e12 / PEAK_FP32})
            rows["multi_rhs_H_k16_fp32c"] = row
            mrows = sample_rows(N, 64, 12)
            U16_np = H2(U16)
            for l in (0, 7, 15):
                check_matvec("multi_rhs_H_k16_fp32c", f"RHS {l}, 64 sampled rows", H.pos, F16_np[l],
                             U16_np[l][mrows], mrows, key=f"error_vs_oracle_rhs{l}")
            # the same 16-RHS product in FP64 (built-in shape: one block of 16
            # on the matrix cores), against two passes of 8 on the vector units
            U16.zero_()
            w64m, km64, _, _ = timed(lambda: rp.matvec_multi(pos, F16, precision=rp.FP64, out=U16), 2, 1)
            sh64 = rp.get_shape(rp.FP64, N, k)
            fv, fm = mat_flop(N, k)
            km64 /= 2
            row64 = {"pair_rhs_per_s": k * N * N / w64m, "ms": w64m * 1e3, "kernel_ms": km64, "shape": sh64,
                     "bound": "mfma", "matrix_tflops": fm / (km64 * 1e-3) / 1e12,
                     "frac_fp64_matrix_peak": fm / (km64 * 1e-3) / 1e12 / PEAK_FP64_MATRIX,
                     "vector_tflops": fv / (km64 * 1e-3) / 1e12,
                     "frac_fp64_vector_peak": fv / (km64 * 1e-3) / 1e12 / PEAK_FP64}
            U64_np = H2(U16)
            rp.set_shape(rp.FP64, N, k, tpl=1, tile=256, kblk=8, sym=0, ipw=4, mat=0)
            wv64, kmv64, _, _ = timed(lambda: rp.matvec_multi(pos, F16, precision=rp.FP64, out=U16), 1, 1)
            rp.reset_shape(rp.FP64, N, k)
            flv = 2 * algorithmic_flop(N, 8, 0)
            row64["vector_kernel"] = {"ms": wv64 * 1e3, "kernel_ms": kmv64, "kblk": 8,
                                      "tflops_alg": flv / (kmv64 * 1e-3) / 1e12,
                                      "frac_fp64_peak": flv / (kmv64 * 1e-3) / 1e12 / PEAK_FP64}
            rows["multi_rhs_H_k16_fp64"] = row64
            for l in (0, 15):
                check_matvec("multi_rhs_H_k16_fp64", f"RHS {l}, 64 sampled rows", H.pos, F16_np[l],
                             U64_np[l][mrows], mrows, key=f"error_vs_oracle_rhs{l}")
            del F16, U16, U16_np, F16_np, U64_np

        # single products on configs 0, 1 and 4 (default launch shapes), both
        # precisions: pairs/s and the pair kernel's share of the call
        if want("product_C0", "product_C1", "product_C4"):
            for cname, cfg in (("C0", wl.config0(seed=0)), ("C1", wl.config1(seed=0)), ("C4", wl.config4(seed=0))):
                fcf_np = wl.gaussian(cfg.pos.shape, 4)
                pcf, fcf = T(cfg.pos), T(fcf_np)
                ucf = torch.empty_like(fcf)
                for prec, pname in ((rp.FP32C, "fp32c"), (rp.FP64, "fp64")):
                    reps = 50 if cfg.N <= 4000 else 10
                    w, km, ln, pr = timed(lambda: rp.matvec(pcf, fcf, precision=prec, out=ucf), reps, 3)
                    shc = rp.get_shape(prec, cfg.N, 1)
                    kms_c = km / max(ln, 1)
                    name = f"product_{cname}_{pname}"
                    rows[name] = {
                        "blobs": cfg.N, "pairs_per_s": cfg.N ** 2 / w, "ms": w * 1e3, "kernel_ms": kms_c,
                        "shape": shc, "tflops_alg": algorithmic_flop(cfg.N, 1, shc["sym"]) / (kms_c * 1e-3) / 1e12}
                    if cfg.N <= 4000:
                        check_matvec(name, f"all {cfg.N} rows", cfg.pos, fcf_np, H2(ucf))
                    else:
                        cr = sample_rows(cfg.N, 256, 13)
                        check_matvec(name, f"256 sampled rows of {cfg.N}", cfg.pos, fcf_np, H2(ucf)[cr], cr)
                del pcf, fcf, ucf

        # batched suspensions (config 3) against per-instance launches
        if want("batched_C3"):
            k = 16
            C3 = wl.config3(seed=0)
            offs = C3.sys_offsets
            S = len(offs) - 1
            F3_np = wl.gaussian((k, C3.N, 3), 3)
            F3 = T(F3_np)
            U3 = torch.empty_like(F3)
            p3 = T(C3.pos)
            nmax = int(max(offs[s + 1] - offs[s] for s in range(S)))
            smax = int(np.argmax(np.diff(offs)))
            rp.autotune(p3[offs[smax]:offs[smax + 1]].contiguous(),
                        F3[:, offs[smax]:offs[smax + 1]].contiguous(), precision=rp.FP32C)
            pairs3 = float(sum(float(offs[s + 1] - offs[s]) ** 2 for s in range(S)))
            wb, _, _, _ = timed(lambda: rp.matvec_batched(p3, offs, F3, precision=rp.FP32C, out=U3), 3, 1)
            slices = [(int(offs[s]), int(offs[s + 1])) for s in range(S)]
            sub = [(p3[a:b].contiguous(), F3[:, a:b].contiguous()) for a, b in slices]

            def per_system_multi():
                for ps, Fs in sub:
                    rp.matvec_multi(ps, Fs, precision=rp.FP32C)

            def per_system_single():
                for ps, Fs in sub:
                    for l in range(k):
                        rp.matvec(ps, Fs[l], precision=rp.FP32C)

            wm, _, _, _ = timed(per_system_multi, 2, 1)
            wsn, _, _, _ = timed(per_system_single, 1, 1)
            rows["batched_C3_k16_fp32c"] = {
                "systems": S, "blobs": C3.N, "largest": nmax, "pair_rhs": k * pairs3,
                "batched_ms": wb * 1e3, "per_system_multi_rhs_ms": wm * 1e3, "per_system_single_rhs_ms": wsn * 1e3,
                "speedup_vs_multi": wm / wb, "speedup_vs_single": wsn / wb,
                "batched_pair_rhs_per_s": k * pairs3 / wb, "shape_largest": rp.get_shape(rp.FP32C, nmax, k)}
            U3_np = H2(U3)
            for s in sorted({0, smax, S // 2, S - 1}):
                b0, b1 = slices[s]
                sr = sample_rows(b1 - b0, 32, 14 + s)
                for l in (0, 15):
                    check_matvec("batched_C3_k16_fp32c", f"system {s} ({b1 - b0} blobs), RHS {l}, 32 sampled rows",
                                 C3.pos[b0:b1], F3_np[l, b0:b1], U3_np[l, b0:b1][sr], sr,
                                 key=f"error_vs_oracle_system{s}_rhs{l}")
            del F3, U3, sub, U3_np

        # Lanczos: 256 boomerangs FP64 tol 1e-6; microrollers FP32C tol 1e-6
        C1 = wl.config1(seed=0)
        W1_np = wl.gaussian(C1.pos.shape, 1)
        pc1, W1 = T(C1.pos), T(W1_np)
        if want("lanczos_C1"):
            rp.lanczos_sqrt(pc1, W1, body_offsets=C1.body_offsets, tol=1e-6)
            sync()
            # the call's time (median of 5), then the product kernel's share
            # from one more call with the library's kernel timing on
            t1s = []
            for _ in range(5):
                t0 = time.perf_counter()
                o1, it1, err1, ok1 = rp.lanczos_sqrt(pc1, W1, body_offsets=C1.body_offsets, tol=1e-6)
                sync()
                t1s.append(time.perf_counter() - t0)
            t1 = float(np.median(t1s))
            rp.profile_enable(True)
            rp.profile_read(True)
            rp.lanczos_sqrt(pc1, W1, body_offsets=C1.body_offsets, tol=1e-6)
            sync()
            kms1, ln1, _ = rp.profile_read(True)
            rp.profile_enable(False)
            rows["lanczos_C1_fp64_tol1e-6"] = {"blobs": C1.N, "iterations": it1, "converged": ok1, "ms": t1 * 1e3,
                                               "ms_min": min(t1s) * 1e3,
                                               "ms_per_iteration": t1 * 1e3 / max(it1, 1),
                                               "product_kernel_ms_per_iteration": kms1 / max(ln1, 1)}
            checks.append({"kind": "lanczos", "row": "lanczos_C1_fp64_tol1e-6", "what": "all 3840 blobs",
                           "name": "C1", "pos": C1.pos, "W": W1_np, "offs": C1.body_offsets, "tol": 1e-6,
                           "got": H2(o1)})
        # Rigid-body mobility solve (GMRES, block-diagonal preconditioner):
        # 256 boomerangs, reference point at the corner blob, random F and T
        if want("rigid_C1"):
            q1_np = C1.pos[C1.body_offsets[:-1]]
            FT1_np = wl.gaussian((len(C1.body_offsets) - 1, 6), 5)
            q1, FT1 = T(q1_np), T(FT1_np)
            for prec, pname in ((rp.FP64, "fp64"), (rp.FP32C, "fp32c")):
                for tol in (1e-3, 1e-6):
                    rp.rigid_solve(pc1, q1, C1.body_offsets, None, FT1, tol=tol, precision=prec)
                    sync()
                    t0 = time.perf_counter()
                    _, Ur, itr, resr, okr = rp.rigid_solve(pc1, q1, C1.body_offsets, None, FT1, tol=tol,
                                                           precision=prec)
                    sync()
                    tr = time.perf_counter() - t0
                    name = f"rigid_C1_{pname}_tol{tol:g}"
                    rows[name] = {"blobs": C1.N, "bodies": len(C1.body_offsets) - 1, "iterations": itr,
                                  "converged": okr, "residual": resr, "ms": tr * 1e3,
                                  "ms_per_iteration": tr * 1e3 / max(itr, 1)}
                    checks.append({"kind": "rigid", "row": name, "what": "U of all 256 bodies", "name": "C1",
                                   "pos": C1.pos, "q": q1_np, "offs": C1.body_offsets, "FT": FT1_np, "tol": tol,
                                   "got": H2(Ur)})
        # Iterations versus suspension size with the paper's boomerang
        # geometry (Sec. II.B: about five at tolerance 1e-3, size-independent)
        if want("rigid_paperlike"):
            for nbody in (256, 1024, 4096):
                PB = wl.paperlike_boomerangs(nbody, seed=2)
                qpb_np = PB.pos[PB.body_offsets[:-1]]
                FTpb_np = wl.gaussian((nbody, 6), 11)
                ppb, qpb = T(PB.pos), T(qpb_np)
                FTpb = T(FTpb_np)
                rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3, precision=rp.FP32C)
                sync()
                t0 = time.perf_counter()
                _, Up, itp, resp, okp = rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3,
                                                      precision=rp.FP32C)
                sync()
                tp = time.perf_counter() - t0
                name = f"rigid_paperlike_{nbody}_fp32c_tol0.001"
                rows[name] = {
                    "blobs": PB.N, "bodies": nbody, "iterations": itp, "converged": okp, "residual": resp,
                    "ms": tp * 1e3, "ms_per_iteration": tp * 1e3 / max(itp, 1)}
                if nbody == 256:
                    checks.append({"kind": "rigid", "row": name, "what": "U of all 256 bodies", "name": "PB256",
                                   "pos": PB.pos, "q": qpb_np, "offs": PB.body_offsets, "FT": FTpb_np, "tol": 1e-3,
                                   "got": H2(Up)})
                else:
                    rows[name]["error_vs_oracle"] = {
                        "rel_l2_vs_oracle": None,
                        "note": "not checked here: the oracle GMRES forms K densely (3N x 6n), too large at this "
                                "size; the 256-body case and the tests cover the solver"}
                del ppb, qpb, FTpb
        # Pseudo-periodic cell (minimum image + 8 images), the paper's dense
        # boomerang suspensions: products and one rigid solve at 1e-3
        if want("periodic_paperlike", "periodic_rigid", "ts_step", "emt_step", "emrfd_step"):
            for nbody in (256, 4096):
                PB = wl.paperlike_boomerangs(nbody, seed=2)
                Lc = 139.8 * math.sqrt(nbody / 256.0)
                fpb_np = wl.gaussian(PB.pos.shape, 12)
                ppb, fpb = T(PB.pos), T(fpb_np)
                if want("periodic_paperlike"):
                    upb = torch.empty_like(fpb)
                    wpp, kpp, lpp, ppp = timed(lambda: rp.matvec(ppb, fpb, precision=rp.FP32C, box=(Lc, Lc),
                                                                 out=upb), 5, 2)
                    name = f"periodic_paperlike_{nbody}_fp32c"
                    rows[name] = {
                        "blobs": PB.N, "cell": Lc, "ms": wpp * 1e3, "kernel_ms": kpp / lpp,
                        "image_pairs_per_s": 9.0 * PB.N ** 2 / wpp,
                        "tflops_alg_sym": 9.0 * algorithmic_flop(PB.N, 1, 1) / (kpp / lpp * 1e-3) / 1e12}
                    pr_ = sample_rows(PB.N, 128, 15)
                    check_matvec(name, f"128 sampled rows of {PB.N}", PB.pos, fpb_np, H2(upb)[pr_], pr_,
                                 box=(Lc, Lc))
                if nbody == 256:
                    if want("periodic_rigid"):
                        qpb_np = PB.pos[PB.body_offsets[:-1]]
                        FTpb_np = wl.gaussian((nbody, 6), 11)
                        qpb, FTpb = T(qpb_np), T(FTpb_np)
                        rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3, precision=rp.FP32C,
                                       box=(Lc, Lc))
                        sync()
                        t0 = time.perf_counter()
                        _, Upr, itp, resp, okp = rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3,
                                                               precision=rp.FP32C, box=(Lc, Lc))
                        sync()
                        name = "periodic_rigid_paperlike_256_fp32c_tol0.001"
                        rows[name] = {
                            "blobs": PB.N, "iterations": itp, "converged": okp, "ms": (time.perf_counter() - t0) * 1e3}
                        checks.append({"kind": "rigid", "row": name, "what": "U of all 256 bodies",
                                       "name": "PB256per", "pos": PB.pos, "q": qpb_np, "offs": PB.body_offsets,
                                       "FT": FTpb_np, "tol": 1e-3, "box": (Lc, Lc), "got": H2(Upr)})
                    # One Trapezoidal Slip step (Alg. 2) in the cell, the paper's
                    # settings for this suspension: tolerance 1e-3, FP32C products,
                    # delta = 1e-3; gravity-like constant force per body
                    # tracking points at the corner blobs, body frames = the current
                    # blob offsets from them (identity orientations)
                    no_oracle = {"rel_l2_vs_oracle": None,
                                 "note": "integrator steps are checked against the oracle's dense steps (same "
                                         "random vectors and forces) in the tests, at 90 blobs; a dense step at "
                                         "3840 blobs is outside this benchmark's time budget"}
                    thb = torch.zeros((nbody, 4), dtype=torch.float64, device=dev)
                    thb[:, 0] = 1.0
                    qb = T(PB.pos[PB.body_offsets[:-1]])
                    refb = T(PB.pos - np.repeat(PB.pos[PB.body_offsets[:-1]], 15, axis=0))
                    Fb = torch.zeros((nbody, 6), dtype=torch.float64, device=dev)
                    Fb[:, 2] = -1.0
                    Wsb, Wnb = T(wl.gaussian(PB.pos.shape, 21)), T(wl.gaussian(PB.pos.shape, 22))
                    if want("ts_step"):
                        stp = rp.TSStep(refb, PB.body_offsets, T(np.full(nbody, 5.0)), 1.0, 0.01, 1e-3, tol=1e-3,
                                        precision=rp.FP32C, box=(Lc, Lc))
                        stp.step(qb, thb, lambda qq, tt, pp: Fb, Wsb, Wnb)
                        sync()
                        t0 = time.perf_counter()
                        for _ in range(3):
                            stp.step(qb, thb, lambda qq, tt, pp: Fb, Wsb, Wnb)
                        sync()
                        rows["ts_step_periodic_paperlike_256_fp32c_tol0.001"] = {
                            "blobs": PB.N, "bodies": nbody, "ms_per_step": (time.perf_counter() - t0) / 3 * 1e3,
                            "iterations_rfd_lanczos_predictor_corrector": stp.iters,
                            "products_per_step": sum(stp.iters) + 2, "error_vs_oracle": dict(no_oracle)}
                    Lpb = T(np.full(nbody, 5.0))
                    Wfb, Wtb = T(wl.gaussian((nbody, 3), 23)), T(wl.gaussian((nbody, 3), 24))
                    for scheme, rname, label in (("emt", "emt_step_periodic_paperlike_256_fp32c_tol0.001",
                                                  "iterations_rfd_lanczos_solve"),
                                                 ("emrfd", "emrfd_step_periodic_paperlike_256_fp32c_tol0.001",
                                                  "iterations_rfd_rfd_lanczos_solve")):
                        if not want(f"{scheme}_step"):
                            continue
                        em = lambda: rp.emt_step(qb, thb, refb, PB.body_offsets, Lpb, Fb, Wfb, Wtb, Wnb,  # noqa
                                                 1.0, 0.01, 1e-3, tol=1e-3, precision=rp.FP32C, box=(Lc, Lc),
                                                 scheme=scheme)
                        em()
                        sync()
                        t0 = time.perf_counter()
                        for _ in range(3):
                            _, _, ite = em()
                        sync()
                        rows[rname] = {
                            "blobs": PB.N, "bodies": nbody, "ms_per_step": (time.perf_counter() - t0) / 3 * 1e3,
                            label: ite, "products_per_step": sum(ite) + (2 if scheme == "emt" else 0),
                            "error_vs_oracle": dict(no_oracle)}
                del ppb, fpb
        if want("lanczos_C2", "product_C2", "rigid_C2"):
            C2 = wl.config2(seed=0)
            W2_np = wl.gaussian(C2.pos.shape, 3)
            pc2, W2 = T(C2.pos), T(W2_np)
            sync()
            t0 = time.perf_counter()
            o32, it2, err2, ok2 = rp.lanczos_sqrt(pc2, W2, body_offsets=C2.body_offsets, tol=1e-6,
                                                  precision=rp.FP32C)
            sync()
            t2 = time.perf_counter() - t0
            o64, it64, _, _ = rp.lanczos_sqrt(pc2, W2, body_offsets=C2.body_offsets, tol=1e-6, precision=rp.FP64)
            u64c2 = rp.matvec(pc2, W2, precision=rp.FP64)
            w2, k2, l2, p2 = timed(lambda: rp.matvec(pc2, W2, precision=rp.FP32C), 2, 1)
            u32c2 = rp.matvec(pc2, W2, precision=rp.FP32C)
            rows["lanczos_C2_fp32c_tol1e-6"] = {
                "blobs": C2.N, "iterations": it2, "converged": ok2, "ms": t2 * 1e3,
                "ms_per_iteration": t2 * 1e3 / max(it2, 1), "iterations_fp64": it64,
                "rel_l2_vs_fp64_gpu": float((o32 - o64).norm() / o64.norm()),
                "error_vs_oracle": {"rel_l2_vs_oracle": None,
                                    "note": "the oracle Lanczos at 196608 blobs is outside the time budget: the "
                                            "FP32C root is compared with the FP64 GPU root (rel_l2_vs_fp64_gpu), "
                                            "and the FP64 GPU product with the oracle on sampled rows "
                                            "(product_C2_fp32c.fp64_error_vs_oracle)"}}
            c2r = sample_rows(C2.N, 128, 16)
            rows["product_C2_fp32c"] = {"blobs": C2.N, "pairs_per_s": C2.N ** 2 / w2, "ms": w2 * 1e3,
                                        "kernel_ms": k2 / max(l2, 1),
                                        "rel_l2_vs_fp64_gpu": float((u32c2 - u64c2).norm() / u64c2.norm())}
            check_matvec("product_C2_fp32c", f"128 sampled rows of {C2.N}", C2.pos, W2_np, H2(u32c2)[c2r], c2r)
            check_matvec("product_C2_fp32c", f"128 sampled rows of {C2.N}", C2.pos, W2_np, H2(u64c2)[c2r], c2r,
                         key="fp64_error_vs_oracle")
            del o32, o64
            nb2 = len(C2.body_offsets) - 1
            q2 = T(C2.pos.reshape(nb2, 12, 3).mean(1))
            FT2 = T(wl.gaussian((nb2, 6), 7))
            rp.rigid_solve(pc2, q2, C2.body_offsets, None, FT2, tol=1e-3, precision=rp.FP32C)
            sync()
            t0 = time.perf_counter()
            _, _, itr2, resr2, okr2 = rp.rigid_solve(pc2, q2, C2.body_offsets, None, FT2, tol=1e-3, precision=rp.FP32C)
            sync()
            tr2 = time.perf_counter() - t0
            rows["rigid_C2_fp32c_tol0.001"] = {
                "blobs": C2.N, "bodies": nb2, "iterations": itr2, "converged": okr2, "residual": resr2,
                "ms": tr2 * 1e3, "ms_per_iteration": tr2 * 1e3 / max(itr2, 1),
                "error_vs_oracle": {"rel_l2_vs_oracle": None,
                                    "note": "not checked here: the oracle GMRES forms K densely; the residual "
                                            "estimate is reported"}}
            del pc2, W2, u64c2, u32c2, q2, FT2

        # VJP on the differentiation workload
        if want("vjp_C4"):
            C4 = wl.config4(seed=0)
            f4_np, g4_np = wl.gaussian(C4.pos.shape, 1), wl.gaussian(C4.pos.shape, 2)
            p4, f4, g4 = T(C4.pos), T(f4_np), T(g4_np)
            vr = sample_rows(C4.N, 128, 17)
            for prec, name, peak in ((rp.FP32C, "fp32c", PEAK_FP32), (rp.FP64, "fp64", PEAK_FP64)):
                w, km, ln, pr = timed(lambda: rp.matvec_vjp(p4, f4, g4, precision=prec), 3, 1)
                gp, gf = rp.matvec_vjp(p4, f4, g4, precision=prec)
                sh = rp.get_shape(prec, C4.N, 1)
                kv = km / max(ln, 1)
                fl = vjp_flop(C4.N, sh["sym"])
                # central differences (h = 1e-4) of g . M(r) f along two random
                # directions, FP64 products
                h = 1e-4
                rng = np.random.default_rng(5)
                fd_worst = 0.0
                for _ in range(2):
                    d = T(rng.standard_normal(C4.pos.shape))
                    lp = float((g4 * rp.matvec(p4 + h * d, f4, precision=rp.FP64)).sum())
                    lm = float((g4 * rp.matvec(p4 - h * d, f4, precision=rp.FP64)).sum())
                    fd = (lp - lm) / (2 * h)
                    fd_worst = max(fd_worst, abs(fd - float((gp * d).sum())) / abs(fd))
                rname = f"vjp_C4_{name}"
                rows[rname] = {"blobs": C4.N, "ms": w * 1e3, "pairs_per_s": C4.N ** 2 / w, "kernel_ms": kv,
                               "shape": sh, "flop_per_launch": fl,
                               "flop_per_unordered_pair": FLOP_VJP_PAIR if sh["sym"] else 2 * FLOP_VJP_SELF,
                               "roofline": {"bound": "alu", "achieved": round(fl / (kv * 1e-3) / 1e12, 3),
                                            "peak": peak, "unit": "TFLOP/s",
                                            "frac": round(fl / (kv * 1e-3) / 1e12 / peak, 4)},
                               "fd_directional_rel_err": fd_worst}
                checks.append({"kind": "vjp", "row": rname, "what": "both gradients, 128 sampled blobs",
                               "pos": C4.pos, "f": f4_np, "g": g4_np, "rows": vr, "got": (H2(gp)[vr], H2(gf)[vr])})
        if want("divergence"):
            D = wl.divergence_config(seed=0)
            pd = T(D.pos)
            w, _, _, _ = timed(lambda: rp.divergence(pd, precision=rp.FP64), 3, 1)
            rows["divergence_500_fp64"] = {"blobs": D.N, "ms": w * 1e3}
            checks.append({"kind": "divergence", "row": "divergence_500_fp64", "what": "all 500 blobs",
                           "pos": D.pos, "got": H2(rp.divergence(pd, precision=rp.FP64))})

    # ---------------------------------------------------------- oracle leg
    top = {}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = oracle_leg(checks, H, args, rows, top)

    rec = {
        "metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1e5 free blobs, x,y~U[0,600], z~U[1.1,6], a=eta=1, f~N(0,1), seed 0 "
                               "(config-0 density at 1e5 blobs)",
                   "N": N, "precision": "FP32 pair terms, compensated FP32 sums, FP64 in/out",
                   "pairs_per_step": N * N},
        "error_vs_oracle": top.get("headline"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        **out,
        "rows": rows,
    }
    if "fp64" in rec:
        rec["fp64"]["error_vs_oracle"] = top.get("fp64_headline")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
