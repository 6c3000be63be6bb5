"""Pins of the oracle's pseudo-periodic mobility (Sec. IV.B: each source blob at
its minimum image along the wall plus the 8 periodic images around it).

Expected values come from the open-domain pair blocks with the images picked
by an independent construction (argmin over a range of shifts instead of
rounding), from the open-domain product in the large-cell limit, and from
the invariances and symmetry the definition implies."""
import math

import numpy as np
import pytest

from paper_1709_02410_amd import workloads as wl


def _cloud(n, L, seed, zlo=1.1, zhi=5.0):
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(0, L, n), rng.uniform(0, L, n), rng.uniform(zlo, zhi, n)])
    return pos


def test_explicit_image_sum(orc):
    """u_i = sum_j sum_{images} M(r_i, image of r_j) f_j with the minimum image
    found by argmin of |dx + n L| over n in [-4, 4] (per axis), for sources
    spread over two cells (so shifts other than 0 and +-1 occur)."""
    Lx, Ly = 11.0, 13.0
    pos = _cloud(14, 1.0, 0)
    pos[:, 0] = np.random.default_rng(1).uniform(-Lx, Lx, 14)
    pos[:, 1] = np.random.default_rng(2).uniform(-Ly, Ly, 14)
    pos[3] = pos[2] + [0.5, -0.3, 0.2]  # an overlapping pair
    f = wl.gaussian(pos.shape, 3)
    u = orc.matvec(pos, f, box=(Lx, Ly))
    ns = np.arange(-4, 5)
    ref = np.zeros_like(u)
    for i in range(len(pos)):
        for j in range(len(pos)):
            d = pos[i] - pos[j]
            nx = ns[np.argmin(np.abs(d[0] + ns * Lx))]
            ny = ns[np.argmin(np.abs(d[1] + ns * Ly))]
            for sx in (-1, 0, 1):
                for sy in (-1, 0, 1):
                    rj = pos[j] - [(nx + sx) * Lx, (ny + sy) * Ly, 0.0]
                    ref[i] += orc.pair_block(pos[i], rj) @ f[j]
    np.testing.assert_allclose(u, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_large_cell_limit_is_the_open_domain(orc):
    pos = _cloud(40, 20.0, 4)
    f = wl.gaussian(pos.shape, 5)
    u_open = orc.matvec(pos, f)
    u_per = orc.matvec(pos, f, box=(1e6, 1.3e6))
    assert np.abs(u_per - u_open).max() <= 1e-12 * np.abs(u_open).max()


def test_translation_and_wrapping_invariance(orc):
    L = (17.0, 15.0)
    pos = _cloud(50, 15.0, 6)
    f = wl.gaussian(pos.shape, 7)
    u = orc.matvec(pos, f, box=L)
    moved = pos + [3.7, -8.2, 0.0]
    np.testing.assert_allclose(orc.matvec(moved, f, box=L), u, rtol=0, atol=1e-13 * np.abs(u).max())
    wrapped = pos.copy()
    wrapped[::3, 0] += 2 * L[0]
    wrapped[1::3, 1] -= 3 * L[1]
    np.testing.assert_allclose(orc.matvec(wrapped, f, box=L), u, rtol=0, atol=1e-12 * np.abs(u).max())


def test_periodic_mobility_symmetric_positive_definite(orc):
    """Paper-like dense boomerang suspension in a small periodic cell."""
    cfg = wl.paperlike_boomerangs(8, seed=3)
    L = math.sqrt(8 / (256.0 / 139.8 ** 2))
    M = orc.dense(cfg.pos, box=(L, L))
    assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    f = wl.gaussian(cfg.pos.shape, 8)
    u = orc.matvec(cfg.pos, f, box=(L, L)).reshape(-1)
    np.testing.assert_allclose(M @ f.reshape(-1), u, rtol=0, atol=1e-13 * np.abs(u).max())


def test_single_blob_sees_its_eight_images(orc):
    """One blob: self block plus its 8 images at (sx Lx, sy Ly), which differ
    from the self block (so the images are included)."""
    L = 6.0
    p = np.array([[1.0, 2.0, 2.5]])
    f = np.array([[0.3, -1.0, 0.7]])
    u = orc.matvec(p, f, box=(L, L))
    ref = orc.pair_block(p[0], p[0]) @ f[0]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            if sx or sy:
                ref += orc.pair_block(p[0], p[0] + [sx * L, sy * L, 0.0]) @ f[0]
    np.testing.assert_allclose(u[0], ref, rtol=1e-14)
    assert np.abs(u[0] - orc.matvec(p, f)[0]).max() > 1e-3 * np.abs(u).max()
