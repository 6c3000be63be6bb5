"""The HIP path's per-pair arithmetic (pair_math.h), compiled for the CPU
with g++, against the FP64 oracle (values) and against central differences
of itself (the hand-derived pair gradient used by the VJP and divergence
kernels).  Runs without a GPU."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")


@pytest.fixture(scope="module")
def pm(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("pm") / "pair_math_host.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-I", HARNESS,
                    os.path.join(HARNESS, "pair_math_host.cpp"), "-o", out], check=True)
    lib = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    for n in ("host_block_f64", "host_block_f32", "host_block2_f64", "host_block2_f32"):
        getattr(lib, n).argtypes = [dp, dp, dp]
    for n in ("host_grad_f64", "host_grad_f32"):
        getattr(lib, n).argtypes = [dp, dp, dp, dp]
    return lib


def _p(x):
    return np.ascontiguousarray(x, dtype=np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _block(pm, d, z, f32=False, written_out=False):
    out = np.empty(9)
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    fn = {(False, False): pm.host_block_f64, (True, False): pm.host_block_f32,
          (False, True): pm.host_block2_f64, (True, True): pm.host_block2_f32}[(f32, written_out)]
    fn(_p(d), _p(z), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out.reshape(3, 3)


def _grad(pm, d, z, v, f32=False):
    out = np.empty(6)
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    (pm.host_grad_f32 if f32 else pm.host_grad_f64)(_p(d), _p(z), _p(v), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def _pairs(rng, n):
    for _ in range(n):
        zi, zj = rng.uniform(1.0, 6.0, 2)
        dxy = rng.uniform(-8, 8, 2) * (0.2 if rng.uniform() < 0.3 else 1.0)
        yield np.array([dxy[0], dxy[1], zi - zj]), np.array([zi, zj])


def test_block_matches_oracle(pm, orc):
    """Unregularised-height blocks (z >= a) of the device formulation equal
    the oracle's blocks (units of mu0) in FP64, and to FP32 rounding in FP32."""
    rng = np.random.default_rng(0)
    for d, z in list(_pairs(rng, 400)) + [(np.zeros(3), np.array([1.7, 1.7]))]:
        ri = np.array([d[0], d[1], z[0]])
        rj = np.array([0.0, 0.0, z[1]])
        ref = orc.pair_block(ri, rj, 1.0, 1.0, 0) * 6 * np.pi
        got = _block(pm, d, z)
        assert np.abs(got - ref).max() <= 2e-15 * max(1.0, np.abs(ref).max()), (d, z)
        got32 = _block(pm, d, z, f32=True)
        assert np.abs(got32 - ref).max() <= 3e-6 * max(1.0, np.abs(ref).max())


def test_written_out_block_matches_oracle(pm, orc):
    """The 3 x 3 block as the matrix-core kernel forms it (pair_block, then
    one contraction per right-hand side) against the oracle's block, at the
    same bars as the applied form, including overlapping and coincident
    pairs."""
    rng = np.random.default_rng(7)
    cases = list(_pairs(rng, 400)) + [(np.zeros(3), np.array([1.7, 1.7])), (np.array([0.3, -0.2, 0.1]),
                                                                             np.array([1.2, 1.1]))]
    for d, z in cases:
        ri = np.array([d[0], d[1], z[0]])
        rj = np.array([0.0, 0.0, z[1]])
        ref = orc.pair_block(ri, rj, 1.0, 1.0, 0) * 6 * np.pi
        got = _block(pm, d, z, written_out=True)
        assert np.abs(got - ref).max() <= 2e-15 * max(1.0, np.abs(ref).max()), (d, z)
        got32 = _block(pm, d, z, f32=True, written_out=True)
        assert np.abs(got32 - ref).max() <= 3e-6 * max(1.0, np.abs(ref).max())
        # and it is the block pair_apply applies, entry for entry in FP64
        assert np.abs(got - _block(pm, d, z)).max() <= 1e-15 * max(1.0, np.abs(ref).max())


def test_pair_gradient_matches_central_differences(pm):
    """d/d(dx, dy, dz, Rz, zz) of a^T M b + a2^T M b2, with (dx, dy, dz, Rz, zz)
    perturbed through the positions: the target moves (dx, dy, dz, Rz, zz)
    together, so each partial is isolated by combining target and source
    moves."""
    rng = np.random.default_rng(1)
    h = 1e-6
    for d, z in _pairs(rng, 300):
        v = rng.standard_normal(12)
        g = _grad(pm, d, z, v)

        def val(dd, zz):
            return _grad(pm, dd, zz, v)[5]

        ex = np.array([h, 0, 0])
        ey = np.array([0, h, 0])
        fd_x = (val(d + ex, z) - val(d - ex, z)) / (2 * h)
        fd_y = (val(d + ey, z) - val(d - ey, z)) / (2 * h)
        # target height: dz, Rz, zz all move
        fd_zi = (val(d + [0, 0, h], z + [h, 0]) - val(d - [0, 0, h], z - [h, 0])) / (2 * h)
        # source height: dz -> -1, Rz -> +1, zz -> z_i
        fd_zj = (val(d - [0, 0, h], z + [0, h]) - val(d + [0, 0, h], z - [0, h])) / (2 * h)
        scale = max(1.0, np.abs(g[:5]).max())
        assert abs(fd_x - g[0]) <= 2e-7 * scale, (d, z, fd_x, g[0])
        assert abs(fd_y - g[1]) <= 2e-7 * scale
        assert abs(fd_zi - (g[2] + g[3] + z[1] * g[4])) <= 2e-7 * scale
        assert abs(fd_zj - (-g[2] + g[3] + z[0] * g[4])) <= 2e-7 * scale


def test_pair_gradient_self_and_overlap(pm):
    """Self pair: no free-part derivative, finite; overlap branch C1 at 2a."""
    v = np.random.default_rng(2).standard_normal(12)
    g = _grad(pm, np.zeros(3), np.array([1.3, 1.3]), v)
    assert np.all(np.isfinite(g))
    g32 = _grad(pm, np.zeros(3), np.array([1.3, 1.3]), v, f32=True)
    assert np.all(np.isfinite(g32))
    assert np.allclose(g32[:5], g[:5], rtol=1e-5, atol=1e-6)
    lo = _grad(pm, np.array([2.0 - 1e-9, 0, 0]), np.array([2.0, 2.0]), v)
    hi = _grad(pm, np.array([2.0 + 1e-9, 0, 0]), np.array([2.0, 2.0]), v)
    assert np.allclose(lo, hi, rtol=1e-7, atol=1e-9)
