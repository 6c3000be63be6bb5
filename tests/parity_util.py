"""Element-wise parity checks shared by the GPU tests.

Every comparison of the HIP path with the FP64 oracle asserts two bounds with
the same bar:

* relative L2 over all compared entries, ``|got - ref|_2 <= bar |ref|_2``
  (the error metric of the precision targets), and
* per entry, ``max_e |got_e - ref_e| <= bar * max_e |ref_e|``, so that one
  bad row (the last partial group, the padded tail, a segment boundary)
  cannot hide under the global norm: with thousands of rows the global bar
  alone would let a single row be off by tens of times the bar.

Both figures are printed, so that a run's log states the observed errors.
"""
from __future__ import annotations

import contextlib

import numpy as np


def errors(got, ref):
    """(relative L2, max entry error / max |ref|) of got against ref."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    d = got - ref
    nref = float(np.linalg.norm(ref))
    mref = float(np.abs(ref).max()) if ref.size else 0.0
    rel = float(np.linalg.norm(d)) / nref if nref > 0 else float(np.linalg.norm(d))
    emax = float(np.abs(d).max()) / mref if mref > 0 else float(np.abs(d).max() if d.size else 0.0)
    return rel, emax


def check(got, ref, bar: float, what: str = "", elem_bar: float | None = None):
    """Assert finite output, relative L2 <= bar and max entry error <=
    elem_bar (default bar) times max |ref|; returns (rel, emax)."""
    got = np.asarray(got, dtype=np.float64)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    rel, emax = errors(got, ref)
    eb = bar if elem_bar is None else elem_bar
    print(f"{what} rel_l2={rel:.3e} max_entry={emax:.3e} (bar {bar:g}, entry bar {eb:g})", flush=True)
    assert rel <= bar, f"{what}: relative L2 {rel:.3e} > {bar:g}"
    assert emax <= eb, f"{what}: max entry error {emax:.3e} > {eb:g} of max |ref|"
    return rel, emax


@contextlib.contextmanager
def krylov_path(rp, N, fused, prec=0):
    """fused: force the symmetric product for this size class, which makes
    the Lanczos and GMRES drivers take their fused four-launch steps (they
    do so whenever the product is symmetric); otherwise the size's default
    shape (below 512 blobs the plain product, whose steps are not fused)."""
    if fused:
        rp.set_shape(prec, N, 1, tpl=1, tile=256, kblk=1, sym=2, ipw=1)
    try:
        yield
    finally:
        if fused:
            rp.reset_shape(prec, N, 1)
