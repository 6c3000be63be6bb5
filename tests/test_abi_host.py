"""C-ABI checks that need no GPU: every declared symbol is exported, argument
validation rejects bad calls before any HIP work, workspace sizing, and the
host tridiagonal square-root solver against a dense eigendecomposition."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1709_02410_amd import rpywall

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpywall.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rpywall.LIB_PATH):
        pytest.skip("librpywall.so not built")
    return rpywall.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rpy_wall|rpyw)_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "rpy_wall_matvec" in names and "rpy_wall_lanczos_sqrt" in names and "rpy_wall_matvec_vjp" in names
    out = subprocess.run(["nm", "-D", "--defined-only", rpywall.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_noalloc_entry_rejects_before_any_gpu_work(lib):
    """The no-allocation product validates on the host like rpy_wall_matvec
    and refuses problems whose workspace exceeds its fixed scratch array
    (RPYW_ENOMEM) before touching the GPU."""
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cap = lib.rpy_wall_noalloc_scratch_bytes()
    assert cap == 32 << 20
    E = rpywall.EINVAL
    assert lib.rpy_wall_matvec_noalloc(None, dummy, dummy, 10, 1.0, 1.0, 0, None) == E
    assert lib.rpy_wall_matvec_noalloc(dummy, dummy, dummy, 0, 1.0, 1.0, 0, None) == E
    assert lib.rpy_wall_matvec_noalloc(dummy, dummy, dummy, 10, -1.0, 1.0, 0, None) == E
    assert lib.rpy_wall_matvec_noalloc(dummy, dummy, dummy, 10, 1.0, 1.0, 5, None) == E
    for prec in (0, 1):
        # the largest N whose product workspace fits, and the refusal above it
        for n in (1, 1000, 3840, 4096):
            assert rpywall.workspace_bytes(rpywall.OP_MATVEC, n, 1, precision=prec) <= cap
        assert rpywall.workspace_bytes(rpywall.OP_MATVEC, 20000, 1, precision=prec) > cap
        assert lib.rpy_wall_matvec_noalloc(dummy, dummy, dummy, 20000, 1.0, 1.0, prec, None) == rpywall.ENOMEM


def test_calibration_kernel_validation(lib):
    dummy = ctypes.c_void_p(0x1000)
    E = rpywall.EINVAL
    assert lib.rpy_wall_calibrate(2, 1, 1, dummy, None) == E
    assert lib.rpy_wall_calibrate(0, 0, 1, dummy, None) == E
    assert lib.rpy_wall_calibrate(0, 1, 0, dummy, None) == E
    assert lib.rpy_wall_calibrate(1, 1, 1, None, None) == E


def test_validation_rejects_before_any_launch(lib):
    E = rpywall.EINVAL
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.rpy_wall_matvec(None, dummy, dummy, 10, 1.0, 1.0, 0, None, 0, None) == E
    assert lib.rpy_wall_matvec(dummy, dummy, dummy, 0, 1.0, 1.0, 0, None, 0, None) == E
    assert lib.rpy_wall_matvec(dummy, dummy, dummy, 10, 0.0, 1.0, 0, None, 0, None) == E
    assert lib.rpy_wall_matvec(dummy, dummy, dummy, 10, 1.0, float("nan"), 0, None, 0, None) == E
    assert lib.rpy_wall_matvec(dummy, dummy, dummy, 10, 1.0, 1.0, 7, None, 0, None) == E
    assert lib.rpy_wall_matvec_multi(dummy, dummy, dummy, 10, 0, 1.0, 1.0, 0, None, 0, None) == E
    bad_offs = (ctypes.c_int64 * 3)(0, 5, 5)
    assert lib.rpy_wall_matvec_batched(dummy, bad_offs, 2, dummy, dummy, 1, 1.0, 1.0, 1, None, 0, None) == E
    offs = (ctypes.c_int64 * 3)(0, 5, 9)
    it = ctypes.c_int32()
    er = ctypes.c_double()
    assert lib.rpy_wall_lanczos_sqrt(dummy, dummy, dummy, 10, 1.0, 1.0, offs, 2, 1e-6, 50, 0, None, 0,
                                     ctypes.byref(it), ctypes.byref(er), None) == E  # offsets end at 9 != N
    big = (ctypes.c_int64 * 2)(0, 43)
    assert lib.rpy_wall_lanczos_sqrt(dummy, dummy, dummy, 43, 1.0, 1.0, big, 1, 1e-6, 50, 0, None, 0,
                                     ctypes.byref(it), ctypes.byref(er), None) == E  # body too large
    assert lib.rpy_wall_lanczos_sqrt(dummy, dummy, dummy, 10, 1.0, 1.0, None, 0, 0.0, 50, 0, None, 0,
                                     ctypes.byref(it), ctypes.byref(er), None) == E  # tol <= 0
    assert lib.rpy_wall_matvec_vjp(dummy, dummy, dummy, None, None, 10, 1.0, 1.0, 0, None, 0, None) == E
    assert lib.rpy_wall_divergence(dummy, None, 10, 1.0, 1.0, 0, None, 0, None) == E
    rig = lambda offs_, nb, N, q=dummy, tol=1e-6, it_=50: lib.rpy_wall_rigid_solve(  # noqa: E731
        dummy, q, offs_, nb, None, None, dummy, dummy, N, 1.0, 1.0, tol, it_, 0, None, 0, ctypes.byref(it),
        ctypes.byref(er), None)
    assert rig(offs, 2, 10) == E        # offsets end at 9 != N
    assert rig(big, 1, 43) == E         # body too large for the per-body factors
    assert rig(offs, 2, 9, q=None) == E  # reference points missing
    assert rig(offs, 0, 9) == E         # no bodies
    assert rig(offs, 2, 9, tol=0.0) == E
    assert rig(offs, 2, 9, it_=0) == E
    assert rig(bad_offs, 2, 5) == E     # empty body
    nan = float("nan")
    assert lib.rpy_wall_matvec_periodic(dummy, dummy, dummy, 10, 1, 1.0, 1.0, 0.0, 5.0, 0, None, 0, None) == E
    assert lib.rpy_wall_matvec_periodic(dummy, dummy, dummy, 10, 1, 1.0, 1.0, 5.0, nan, 0, None, 0, None) == E
    assert lib.rpy_wall_lanczos_sqrt_periodic(dummy, dummy, dummy, 10, 1.0, 1.0, -1.0, 5.0, None, 0, 1e-6, 50, 0,
                                              None, 0, ctypes.byref(it), ctypes.byref(er), None) == E
    assert lib.rpy_wall_rigid_solve_periodic(dummy, dummy, offs, 2, None, None, dummy, dummy, 9, 1.0, 1.0, 5.0,
                                             float("inf"), 1e-6, 50, 0, None, 0, ctypes.byref(it),
                                             ctypes.byref(er), None) == E
    i3 = (ctypes.c_int32 * 3)()
    ts = lambda dt=0.1, delta=1e-3, kT=1.0, Lp=dummy, st=ctypes.c_void_p(0x100000), sb=1 << 30: (  # noqa: E731
        lib.rpy_wall_ts_predict(dummy, dummy, dummy, offs, 2, 9, Lp, dummy, dummy, dummy, kT, dt, delta, 1.0, 1.0,
                                0.0, 0.0, 1e-3, 50, 0, dummy, dummy, dummy, st, sb, None, 0, i3, None))
    assert ts(dt=0.0) == E
    assert ts(delta=-1.0) == E
    assert ts(kT=-1.0) == E
    assert ts(Lp=None) == E
    assert ts(st=ctypes.c_void_p(0x100008)) == E  # state not 256-byte aligned
    assert ts(sb=16) == E                         # state too small
    assert lib.rpy_wall_ts_correct(dummy, dummy, dummy, dummy, dummy, offs, 2, 9, dummy, None, 0.1, 1.0, 1.0, 0.0,
                                   0.0, 1e-3, 50, 0, dummy, dummy, None, 0, ctypes.byref(it), None) == E
    assert lib.rpy_wall_body_move(dummy, dummy, None, 0.1, 2, dummy, dummy, None) == E
    assert lib.rpy_wall_emt_step(dummy, dummy, dummy, offs, 2, 9, dummy, dummy, dummy, None, dummy, 1.0, 0.1, 1e-3,
                                 1.0, 1.0, 0.0, 0.0, 1e-3, 50, 0, dummy, dummy, None, 0, i3, None) == E  # Wt missing
    assert lib.rpy_wall_emt_step(dummy, dummy, dummy, offs, 2, 9, dummy, dummy, dummy, dummy, dummy, 1.0, 0.1, 1e-3,
                                 1.0, 1.0, 5.0, 0.0, 1e-3, 50, 0, dummy, dummy, None, 0, i3, None) == E  # half a cell
    assert lib.rpy_wall_body_blobs(dummy, dummy, dummy, bad_offs, 2, dummy, 5, None, 0, None) == E
    # misaligned caller workspace
    assert lib.rpy_wall_matvec(dummy, dummy, dummy, 10, 1.0, 1.0, 0, ctypes.c_void_p(0x1001), 1 << 20,
                               None) == E


def test_workspace_sizes(lib):
    for op in range(7):
        assert rpywall.workspace_bytes(op, 1000, 4, 50, 10 if op in (1, 5, 6) else 0, 1) > 0
    assert rpywall.workspace_bytes(5, 1000, 1, 50, 0) == 0  # rigid solve needs bodies
    assert lib.rpy_wall_workspace_bytes(0, 0, 1, 0, 0, 0) == 0
    assert lib.rpy_wall_workspace_bytes(9, 10, 1, 0, 0, 0) == 0
    small = rpywall.workspace_bytes(0, 1000, 1)
    assert rpywall.workspace_bytes(0, 100000, 1) > small
    assert rpywall.workspace_bytes(2, 1000, 1, 100, 0) > rpywall.workspace_bytes(2, 1000, 1, 10, 0)
    for s in (0, 1, -1, -2, -3, -4, 99):
        assert lib.rpyw_strerror(s)


@pytest.mark.parametrize("k", [1, 2, 5, 30, 120, 250])
def test_tridiagonal_root_coefficients(lib, k):
    """beta0 T^{1/2} e1 from the host solver (quadrature for SPD T) against
    numpy's eigendecomposition."""
    rng = np.random.default_rng(k)
    alpha = rng.uniform(0.5, 2.0, k)
    beta = rng.uniform(0.01, 0.4, max(k - 1, 0))
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    lam, Q = np.linalg.eigh(T)
    ref = 1.7 * Q @ (np.sqrt(np.clip(lam, 0, None)) * Q[0])
    got = rpywall.tridiag_sqrt_coeffs(alpha, beta, 1.7)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("case", ["split", "clustered", "graded", "lanczos_like", "tiny_offdiag"])
def test_tridiagonal_root_structured(lib, case):
    """The implicit QR solver on matrices that exercise deflation and
    shifts: a zero off-diagonal in the middle, clustered and graded
    eigenvalues, the tridiagonal of a Lanczos run on an SPD matrix, and
    off-diagonals at rounding level."""
    rng = np.random.default_rng(7)
    k = 60
    if case == "split":
        alpha = rng.uniform(0.5, 2.0, k)
        beta = rng.uniform(0.01, 0.4, k - 1)
        beta[k // 2] = 0.0
    elif case == "clustered":
        alpha = 1.0 + 1e-9 * rng.standard_normal(k)
        beta = 1e-7 * rng.uniform(0.5, 1.0, k - 1)
    elif case == "graded":
        alpha = np.logspace(0, -6, k)
        beta = 0.3 * np.sqrt(alpha[:-1] * alpha[1:])
    elif case == "lanczos_like":
        A = rng.standard_normal((200, 200))
        A = A @ A.T / 200 + 0.1 * np.eye(200)
        v = rng.standard_normal(200)
        V = [v / np.linalg.norm(v)]
        alpha, beta = [], []
        for j in range(k):
            w = A @ V[-1]
            alpha.append(V[-1] @ w)
            for u in V:
                w -= (u @ w) * u
            for u in V:
                w -= (u @ w) * u
            if j < k - 1:
                beta.append(np.linalg.norm(w))
                V.append(w / beta[-1])
        alpha, beta = np.array(alpha), np.array(beta)
    else:
        alpha = rng.uniform(0.5, 2.0, k)
        beta = 1e-17 * rng.uniform(0.5, 1.0, k - 1)
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    lam, Q = np.linalg.eigh(T)
    ref = 1.3 * Q @ (np.sqrt(np.clip(lam, 0, None)) * Q[0])
    got = rpywall.tridiag_sqrt_coeffs(alpha, beta, 1.3)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), case


@pytest.mark.parametrize("kappa", [1e1, 1e3, 1e6, 1e9, 1e12, 1e14])
@pytest.mark.parametrize("k", [5, 40, 150])
def test_tridiagonal_root_across_conditioning(lib, kappa, k):
    """The Lanczos tridiagonal of a diagonal SPD matrix with spectrum in
    [1 / kappa, 1] (both ends present): the host square root (quadrature while
    hi / lo <= 1e8, the eigendecomposition beyond) against numpy's eigh."""
    rng = np.random.default_rng(int(np.log10(kappa)) * 1000 + k)
    lam = np.exp(rng.uniform(np.log(1.0 / kappa), 0.0, 400))
    lam[0], lam[1] = 1.0 / kappa, 1.0
    v = rng.standard_normal(400)
    V = [v / np.linalg.norm(v)]
    alpha, beta = [], []
    for j in range(k):
        w = lam * V[-1]
        alpha.append(V[-1] @ w)
        w -= alpha[-1] * V[-1]
        for _ in range(2):
            for u in V:
                w -= (u @ w) * u
        if j < k - 1:
            beta.append(np.linalg.norm(w))
            V.append(w / beta[-1])
    alpha, beta = np.array(alpha), np.array(beta)
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    ev, Q = np.linalg.eigh(T)
    ref = Q @ (np.sqrt(np.clip(ev, 0, None)) * Q[0])
    got = rpywall.tridiag_sqrt_coeffs(alpha, beta, 1.0)
    # both computations are backward stable; with eigenvalues down to 1e-8
    # of the largest (k = 150, kappa >= 1e9) they differ by up to about
    # 5e-13 of the largest coefficient, whichever host method runs
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tridiagonal_root_clamps_negative_eigenvalues(lib):
    alpha = np.array([1.0, -3.0, 0.5])
    beta = np.array([0.2, 0.1])
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    lam, Q = np.linalg.eigh(T)
    ref = Q @ (np.sqrt(np.clip(lam, 0, None)) * Q[0])
    assert np.allclose(rpywall.tridiag_sqrt_coeffs(alpha, beta, 1.0), ref, atol=1e-14)
    with pytest.raises(rpywall.RpywError):
        rpywall.tridiag_sqrt_coeffs(np.array([1.0, np.nan]), np.array([0.1]), 1.0)


def test_launch_shape_validation_and_defaults(lib):
    """Shape overrides: sym 0, 1 (groups of 256) and 2 (groups of 64) are
    accepted, other values and symmetric blocks wider than 4 are not; the
    built-in choice takes groups of 64 for small single-RHS problems."""
    E = rpywall.EINVAL
    assert lib.rpy_wall_set_shape(1, 5000, 1, 1, 256, 1, 3, 1, 0) == E
    assert lib.rpy_wall_set_shape(1, 5000, 1, 1, 256, 8, 2, 1, 0) == E
    assert lib.rpy_wall_set_shape(1, 5000, 1, 1, 256, 1, -1, 1, 0) == E
    # the matrix-core contraction: blocks of 8 or 16 right-hand sides; FP64
    # blocks of 16 only there
    assert lib.rpy_wall_set_shape(1, 5000, 16, 1, 64, 4, 0, 4, 1) == E
    assert lib.rpy_wall_set_shape(1, 5000, 16, 1, 64, 16, 0, 4, 2) == E
    assert lib.rpy_wall_set_shape(0, 5000, 16, 1, 64, 16, 0, 4, 0) == E
    for prec in (0, 1):
        for mat in (0, 1):
            kb = 16 if (prec == 1 or mat) else 8
            rpywall.set_shape(prec, 5000, 16, tpl=1, tile=64, kblk=kb, sym=0, ipw=4, mat=mat)
            assert rpywall.get_shape(prec, 5000, 16) == dict(tpl=1, tile=64, kblk=kb, sym=0, ipw=4, mat=mat)
        rpywall.reset_shape(prec, 5000, 16)
    assert rpywall.get_shape(1, 100000, 16)["mat"] == 1
    assert rpywall.get_shape(1, 100000, 8)["mat"] == 1
    assert rpywall.get_shape(1, 100000, 4)["mat"] == 0
    assert rpywall.get_shape(0, 100000, 16)["mat"] == 1 and rpywall.get_shape(0, 100000, 16)["kblk"] == 16
    assert rpywall.get_shape(0, 100000, 8)["mat"] == 0 and rpywall.get_shape(0, 100000, 8)["kblk"] == 8
    for sym in (0, 1, 2):
        rpywall.set_shape(1, 5000, 1, tpl=1, tile=256, kblk=1, sym=sym, ipw=2)
        assert rpywall.get_shape(1, 5000, 1)["sym"] == sym
    rpywall.reset_shape(1, 5000, 1)
    assert rpywall.get_shape(1, 3840, 1)["sym"] == 2
    assert rpywall.get_shape(0, 100000, 1)["sym"] == 1
    assert rpywall.get_shape(1, 1000, 1)["sym"] == 2
    assert rpywall.get_shape(1, 300, 1)["sym"] == 0
    assert rpywall.get_shape(1, 3840, 4)["sym"] == 0
