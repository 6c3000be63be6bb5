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
# Algorithmic FLOPs per pair of the product kernel (FMA = 2, rsqrt = 1,
# compare/select = 0, precision bookkeeping not counted): 84 shared by all
# right-hand sides + 24 per right-hand side.
FLOP_PAIR_SHARED = 84
FLOP_PAIR_RHS = 24
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_kernel_traffic.json")
KERNEL_SOURCES = ["pair_kernels.hip", "pair_math.h", "records.h", "sym_pairs.h"]


def algorithmic_flop(N: int, k: int, sym: int) -> float:
    """Algorithmic FLOPs of one product of N blobs and k RHS.  The plain
    kernel evaluates every ordered pair (84 + 24 k each); the symmetric
    kernel evaluates each unordered pair once and applies it both ways
    (84 + 48 k), self pairs once (84 + 24 k)."""
    n = float(N)
    if sym:
        return n * (n - 1) / 2 * (FLOP_PAIR_SHARED + 2 * k * FLOP_PAIR_RHS) + n * (FLOP_PAIR_SHARED + k * FLOP_PAIR_RHS)
    return n * n * (FLOP_PAIR_SHARED + k * FLOP_PAIR_RHS)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--headline-only", action="store_true", help="time only the headline product")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    def sync():
        torch.cuda.synchronize()

    def timed(fn, steps, warmup):
        """Wall time per call over `steps` calls and the library-recorded
        pair-kernel time (HIP events on the launch stream)."""
        for _ in range(warmup):
            fn()
        sync()
        rp.profile_enable(True)
        rp.profile_read(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        sync()
        wall = (time.perf_counter() - t0) / steps
        kms, launches, pairs = rp.profile_read(True)
        rp.profile_enable(False)
        return wall, kms, launches, pairs

    def want(*names):
        """Whether any of these rows is selected (all are without --only)."""
        return not args.only or any(o in n for o in args.only for n in names)

    out = {}
    # ---------------------------------------------------------- headline
    H = wl.headline(seed=0)
    N = H.N
    pos = T(H.pos)
    f = T(wl.gaussian(H.pos.shape, 1))
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
    kname = ("sym_kernel<float,1> (each unordered pair once, both directions)" if shape32["sym"]
             else f"pair_kernel<float,1,{shape32['tpl']},{shape32['tile']}>")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32, 4), "traffic": traffic,
                "kernel": kname + ", FP32 pair terms, TwoSum sums", "shape": shape32,
                "kernel_ms_avg": round(kavg, 4), "flop_per_launch": flop_launch,
                "flop_per_ordered_pair": round(flop_launch / (float(N) * N), 2)}

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        out["calib_copy_bytes"] = src.numel() * 8

    # FP64 product on the same input
    step64 = lambda: rp.matvec(pos, f, precision=rp.FP64, out=vel)  # noqa: E731
    w64, k64, l64, p64 = timed(step64, max(3, args.steps // 2), 1)
    shape64 = rp.get_shape(rp.FP64, N, 1)
    a64 = algorithmic_flop(N, 1, shape64["sym"]) / (k64 / l64 * 1e-3) / 1e12
    out["fp64"] = {"value": N * N / w64, "unit": "pair interactions/s", "ms_per_step": w64 * 1e3,
                   "kernel_ms_avg": k64 / l64, "shape": shape64,
                   "roofline": {"bound": "alu", "achieved": round(a64, 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
                                "frac": round(a64 / PEAK_FP64, 4)}}

    rows = {}
    if not args.headline_only:
        # 16-RHS product on the headline geometry
        if want("multi_rhs"):
            k = 16
            F16 = T(wl.gaussian((k, N, 3), 2))
            U16 = torch.empty_like(F16)
            rp.autotune(pos, F16, precision=rp.FP32C)
            w, km, ln, pr = timed(lambda: rp.matvec_multi(pos, F16, precision=rp.FP32C, out=U16), 3, 1)
            sh16 = rp.get_shape(rp.FP32C, N, k)
            fl = sum(algorithmic_flop(N, min(sh16["kblk"], k - k0), sh16["sym"]) for k0 in range(0, k, sh16["kblk"]))
            call_ms = km / 3  # kernel time of one call (three timed calls)
            rows["multi_rhs_H_k16_fp32c"] = {"pair_rhs_per_s": k * N * N / w, "ms": w * 1e3, "shape": sh16,
                                             "tflops_alg": fl / (call_ms * 1e-3) / 1e12,
                                             "frac_fp32_peak": fl / (call_ms * 1e-3) / 1e12 / PEAK_FP32}
            del F16, U16

        # single products on configs 0, 1 and 4 (default launch shapes), both
        # precisions: pairs/s and the pair kernel's share of the call
        if want("product_C0", "product_C1", "product_C4"):
            for cname, cfg in (("C0", wl.config0(seed=0)), ("C1", wl.config1(seed=0)), ("C4", wl.config4(seed=0))):
                pcf, fcf = T(cfg.pos), T(wl.gaussian(cfg.pos.shape, 4))
                ucf = torch.empty_like(fcf)
                for prec, pname in ((rp.FP32C, "fp32c"), (rp.FP64, "fp64")):
                    reps = 50 if cfg.N <= 4000 else 10
                    w, km, ln, pr = timed(lambda: rp.matvec(pcf, fcf, precision=prec, out=ucf), reps, 3)
                    shc = rp.get_shape(prec, cfg.N, 1)
                    kms = km / max(ln, 1)
                    rows[f"product_{cname}_{pname}"] = {
                        "blobs": cfg.N, "pairs_per_s": cfg.N ** 2 / w, "ms": w * 1e3, "kernel_ms": kms, "shape": shc,
                        "tflops_alg": algorithmic_flop(cfg.N, 1, shc["sym"]) / (kms * 1e-3) / 1e12}
                del pcf, fcf, ucf

        # batched suspensions (config 3) against per-instance launches
        if want("batched_C3"):
            C3 = wl.config3(seed=0)
            offs = C3.sys_offsets
            S = len(offs) - 1
            F3 = T(wl.gaussian((k, C3.N, 3), 3))
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
                "batched_pair_rhs_per_s": k * pairs3 / wb}
            del F3, U3, sub

        # Lanczos: 256 boomerangs FP64 tol 1e-6; microrollers FP32C tol 1e-6
        C1 = wl.config1(seed=0)
        pc1, W1 = T(C1.pos), T(wl.gaussian(C1.pos.shape, 1))
        if want("lanczos_C1"):
            rp.lanczos_sqrt(pc1, W1, body_offsets=C1.body_offsets, tol=1e-6)
            sync()
            t0 = time.perf_counter()
            _, it1, err1, ok1 = rp.lanczos_sqrt(pc1, W1, body_offsets=C1.body_offsets, tol=1e-6)
            sync()
            t1 = time.perf_counter() - t0
            rows["lanczos_C1_fp64_tol1e-6"] = {"blobs": C1.N, "iterations": it1, "converged": ok1, "ms": t1 * 1e3,
                                               "ms_per_iteration": t1 * 1e3 / max(it1, 1)}
        # Rigid-body mobility solve (GMRES, block-diagonal preconditioner):
        # 256 boomerangs, reference point at the corner blob, random F and T
        if want("rigid_C1"):
            q1 = T(C1.pos[C1.body_offsets[:-1]])
            FT1 = T(wl.gaussian((len(C1.body_offsets) - 1, 6), 5))
            for prec, pname in ((rp.FP64, "fp64"), (rp.FP32C, "fp32c")):
                for tol in (1e-3, 1e-6):
                    rp.rigid_solve(pc1, q1, C1.body_offsets, None, FT1, tol=tol, precision=prec)
                    sync()
                    t0 = time.perf_counter()
                    _, _, itr, resr, okr = rp.rigid_solve(pc1, q1, C1.body_offsets, None, FT1, tol=tol, precision=prec)
                    sync()
                    tr = time.perf_counter() - t0
                    rows[f"rigid_C1_{pname}_tol{tol:g}"] = {"blobs": C1.N, "bodies": len(C1.body_offsets) - 1,
                                                            "iterations": itr, "converged": okr, "residual": resr,
                                                            "ms": tr * 1e3, "ms_per_iteration": tr * 1e3 / max(itr, 1)}
        # Iterations versus suspension size with the paper's boomerang
        # geometry (Sec. II.B: about five at tolerance 1e-3, size-independent)
        if want("rigid_paperlike"):
            for nbody in (256, 1024, 4096):
                PB = wl.paperlike_boomerangs(nbody, seed=2)
                ppb, qpb = T(PB.pos), T(PB.pos[PB.body_offsets[:-1]])
                FTpb = T(wl.gaussian((nbody, 6), 11))
                rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3, precision=rp.FP32C)
                sync()
                t0 = time.perf_counter()
                _, _, itp, resp, okp = rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3,
                                                     precision=rp.FP32C)
                sync()
                tp = time.perf_counter() - t0
                rows[f"rigid_paperlike_{nbody}_fp32c_tol0.001"] = {
                    "blobs": PB.N, "bodies": nbody, "iterations": itp, "converged": okp, "residual": resp,
                    "ms": tp * 1e3, "ms_per_iteration": tp * 1e3 / max(itp, 1)}
                del ppb, qpb, FTpb
        # Pseudo-periodic cell (minimum image + 8 images), the paper's dense
        # boomerang suspensions: products and one rigid solve at 1e-3
        if want("periodic_paperlike", "periodic_rigid", "ts_step", "emt_step", "emrfd_step"):
            for nbody in (256, 4096):
                PB = wl.paperlike_boomerangs(nbody, seed=2)
                Lc = 139.8 * math.sqrt(nbody / 256.0)
                ppb, fpb = T(PB.pos), T(wl.gaussian(PB.pos.shape, 12))
                if want("periodic_paperlike"):
                    wpp, kpp, lpp, ppp = timed(lambda: rp.matvec(ppb, fpb, precision=rp.FP32C, box=(Lc, Lc)), 5, 2)
                    rows[f"periodic_paperlike_{nbody}_fp32c"] = {
                        "blobs": PB.N, "cell": Lc, "ms": wpp * 1e3, "kernel_ms": kpp / lpp,
                        "image_pairs_per_s": 9.0 * PB.N ** 2 / wpp,
                        "tflops_alg_sym": 9.0 * algorithmic_flop(PB.N, 1, 1) / (kpp / lpp * 1e-3) / 1e12}
                if nbody == 256:
                    if want("periodic_rigid"):
                        qpb = T(PB.pos[PB.body_offsets[:-1]])
                        FTpb = T(wl.gaussian((nbody, 6), 11))
                        rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3, precision=rp.FP32C,
                                       box=(Lc, Lc))
                        sync()
                        t0 = time.perf_counter()
                        _, _, itp, resp, okp = rp.rigid_solve(ppb, qpb, PB.body_offsets, None, FTpb, tol=1e-3,
                                                             precision=rp.FP32C, box=(Lc, Lc))
                        sync()
                        rows["periodic_rigid_paperlike_256_fp32c_tol0.001"] = {
                            "blobs": PB.N, "iterations": itp, "converged": okp, "ms": (time.perf_counter() - t0) * 1e3}
                if nbody == 256:
                    # One Trapezoidal Slip step (Alg. 2) in the cell, the paper's
                    # settings for this suspension: tolerance 1e-3, FP32C products,
                    # delta = 1e-3; gravity-like constant force per body
                    # tracking points at the corner blobs, body frames = the current
                    # blob offsets from them (identity orientations)
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
                            "products_per_step": sum(stp.iters) + 2}
                    Lpb = T(np.full(nbody, 5.0))
                    Wfb, Wtb = T(wl.gaussian((nbody, 3), 23)), T(wl.gaussian((nbody, 3), 24))
                    if want("emt_step"):
                        emt = lambda: rp.emt_step(qb, thb, refb, PB.body_offsets, Lpb, Fb, Wfb, Wtb, Wnb,  # noqa
                                                  1.0, 0.01, 1e-3, tol=1e-3, precision=rp.FP32C, box=(Lc, Lc))
                        emt()
                        sync()
                        t0 = time.perf_counter()
                        for _ in range(3):
                            _, _, ite = emt()
                        sync()
                        rows["emt_step_periodic_paperlike_256_fp32c_tol0.001"] = {
                            "blobs": PB.N, "bodies": nbody, "ms_per_step": (time.perf_counter() - t0) / 3 * 1e3,
                            "iterations_rfd_lanczos_solve": ite, "products_per_step": sum(ite) + 2}
                    if want("emrfd_step"):
                        emr = lambda: rp.emt_step(qb, thb, refb, PB.body_offsets, Lpb, Fb, Wfb, Wtb, Wnb,  # noqa
                                                  1.0, 0.01, 1e-3, tol=1e-3, precision=rp.FP32C, box=(Lc, Lc),
                                                  scheme="emrfd")
                        emr()
                        sync()
                        t0 = time.perf_counter()
                        for _ in range(3):
                            _, _, ite = emr()
                        sync()
                        rows["emrfd_step_periodic_paperlike_256_fp32c_tol0.001"] = {
                            "blobs": PB.N, "bodies": nbody, "ms_per_step": (time.perf_counter() - t0) / 3 * 1e3,
                            "iterations_rfd_rfd_lanczos_solve": ite, "products_per_step": sum(ite)}
                del ppb, fpb
        if want("lanczos_C2", "product_C2", "rigid_C2"):
            C2 = wl.config2(seed=0)
            pc2, W2 = T(C2.pos), T(wl.gaussian(C2.pos.shape, 3))
            sync()
            t0 = time.perf_counter()
            _, it2, err2, ok2 = rp.lanczos_sqrt(pc2, W2, body_offsets=C2.body_offsets, tol=1e-6,
                                                precision=rp.FP32C)
            sync()
            t2 = time.perf_counter() - t0
            u64c2 = rp.matvec(pc2, W2, precision=rp.FP64)
            w2, k2, l2, p2 = timed(lambda: rp.matvec(pc2, W2, precision=rp.FP32C), 2, 1)
            u32c2 = rp.matvec(pc2, W2, precision=rp.FP32C)
            rows["lanczos_C2_fp32c_tol1e-6"] = {"blobs": C2.N, "iterations": it2, "converged": ok2, "ms": t2 * 1e3,
                                                "ms_per_iteration": t2 * 1e3 / max(it2, 1)}
            rows["product_C2_fp32c"] = {"blobs": C2.N, "pairs_per_s": C2.N ** 2 / w2, "ms": w2 * 1e3,
                                        "rel_l2_vs_fp64": float((u32c2 - u64c2).norm() / u64c2.norm())}
            nb2 = len(C2.body_offsets) - 1
            q2 = T(C2.pos.reshape(nb2, 12, 3).mean(1))
            FT2 = T(wl.gaussian((nb2, 6), 7))
            rp.rigid_solve(pc2, q2, C2.body_offsets, None, FT2, tol=1e-3, precision=rp.FP32C)
            sync()
            t0 = time.perf_counter()
            _, _, itr2, resr2, okr2 = rp.rigid_solve(pc2, q2, C2.body_offsets, None, FT2, tol=1e-3, precision=rp.FP32C)
            sync()
            tr2 = time.perf_counter() - t0
            rows["rigid_C2_fp32c_tol0.001"] = {"blobs": C2.N, "bodies": nb2, "iterations": itr2, "converged": okr2,
                                               "residual": resr2, "ms": tr2 * 1e3,
                                               "ms_per_iteration": tr2 * 1e3 / max(itr2, 1)}
            del pc2, W2, u64c2, u32c2, q2, FT2

        # VJP on the differentiation workload
        if want("vjp_C4"):
            C4 = wl.config4(seed=0)
            p4, f4, g4 = T(C4.pos), T(wl.gaussian(C4.pos.shape, 1)), T(wl.gaussian(C4.pos.shape, 2))
            for prec, name in ((rp.FP32C, "fp32c"), (rp.FP64, "fp64")):
                w, km, ln, pr = timed(lambda: rp.matvec_vjp(p4, f4, g4, precision=prec), 3, 1)
                rows[f"vjp_C4_{name}"] = {"blobs": C4.N, "ms": w * 1e3, "pairs_per_s": C4.N ** 2 / w,
                                          "kernel_ms": km / ln}
        if want("divergence"):
            D = wl.divergence_config(seed=0)
            pd = T(D.pos)
            w, _, _, _ = timed(lambda: rp.divergence(pd, precision=rp.FP64), 3, 1)
            rows["divergence_500_fp64"] = {"blobs": D.N, "ms": w * 1e3}

    # ---------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        orc.build()
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        nthreads = max(1, min(nthreads, os.cpu_count() or 1))
        fh = wl.gaussian(H.pos.shape, 1)
        rng = np.random.default_rng(0)
        probe = rng.choice(N, 4 * nthreads, replace=False)
        t0 = time.perf_counter()
        orc.matvec(H.pos, fh, rows=probe, nthreads=nthreads)
        rate = len(probe) * N / (time.perf_counter() - t0)
        nrows = int(min(N, max(len(probe), args.cpu_seconds * rate / N)))
        rows_s = rng.choice(N, nrows, replace=False)
        t0 = time.perf_counter()
        orc.matvec(H.pos, fh, rows=rows_s, nthreads=nthreads)
        dt = time.perf_counter() - t0
        cpu = {"value": nrows * N / dt, "unit": "pair interactions/s", "cores": nthreads, "kind": "oracle",
               "sample": f"{nrows} random target rows x all {N} sources of the headline product, FP64, "
                         f"{dt:.1f} s (C++ double loop, OpenMP)"}

    rec = {
        "metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1e5 free blobs, x,y~U[0,600], z~U[1.1,6], a=eta=1, f~N(0,1), seed 0 "
                               "(config-0 density at 1e5 blobs)",
                   "N": N, "precision": "FP32 pair terms, compensated FP32 sums, FP64 in/out",
                   "pairs_per_step": N * N},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **out,
        "rows": rows,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
