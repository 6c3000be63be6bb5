"""Seeded synthetic blob configurations.

This module only builds inputs: blob positions, body layouts, forces and
Gaussian vectors.  It contains none of the mobility arithmetic, so both the
FP64 CPU oracle (through the tests) and the HIP path can consume its output
without sharing any method code.

The geometries follow the particle models of the paper's results section:
15-blob L-shaped boomerangs with two 7-blob arms and a shared corner blob
(Sec. IV, boomerang model), and 12-blob microroller spheres whose blobs sit
on the vertices of an icosahedron (Sec. IV, microroller suspensions).  All
lengths are in units of the blob radius ``a`` unless ``a`` is passed.

Every generator takes an integer seed and uses numpy's PCG64
``default_rng``; results are float64 arrays of shape (N, 3) (row-major,
x/y/z per blob), plus int64 body offsets where bodies exist.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Config", "uniform_slab", "gaussian", "boomerang_frame", "icosahedron_frame",
    "boomerang_suspension", "microroller_suspension", "config0", "config1",
    "config2", "config3", "config4", "divergence_config", "headline",
    "paperlike_boomerangs",
]


@dataclass
class Config:
    """A synthetic blob configuration.

    pos: (N, 3) float64 blob centres.
    body_offsets: int64 [n_bodies + 1] or None (free blobs).
    sys_offsets: int64 [S + 1] for batched independent systems, else None.
    meta: free-form description of the recipe.
    """
    name: str
    pos: np.ndarray
    body_offsets: np.ndarray | None = None
    sys_offsets: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.pos.shape[0])


def gaussian(shape, seed: int) -> np.ndarray:
    """iid N(0,1) float64 array (forces, Lanczos seeds W, upstream gradients)."""
    return np.random.default_rng(seed).standard_normal(shape)


def uniform_slab(N: int, box: float, zlo: float, zhi: float, seed: int, a: float = 1.0) -> np.ndarray:
    """N blobs with x, y ~ U[0, box] and z ~ U[zlo, zhi] (all times a)."""
    rng = np.random.default_rng(seed)
    pos = np.empty((N, 3))
    pos[:, 0] = rng.uniform(0.0, box, N)
    pos[:, 1] = rng.uniform(0.0, box, N)
    pos[:, 2] = rng.uniform(zlo, zhi, N)
    return pos * a


def config0(seed: int = 0) -> Config:
    """1000 free blobs, x, y in [0,60]^2, z in [1.1, 6] (a = 1)."""
    return Config("C0", uniform_slab(1000, 60.0, 1.1, 6.0, seed),
                  meta={"recipe": "x,y~U[0,60], z~U[1.1,6], N=1000", "seed": seed})


def headline(seed: int = 0, N: int = 100_000) -> Config:
    """Config-0 distribution at 1e5 blobs with matched areal density (box 600)."""
    box = 60.0 * math.sqrt(N / 1000.0)
    return Config("H", uniform_slab(N, box, 1.1, 6.0, seed),
                  meta={"recipe": f"x,y~U[0,{box:g}], z~U[1.1,6], N={N}", "seed": seed})


def config4(seed: int = 0, N: int = 50_000) -> Config:
    """Differentiation workload: 5e4 blobs in a 300 x 300 box, z in [1.1, 6]."""
    return Config("C4", uniform_slab(N, 300.0, 1.1, 6.0, seed),
                  meta={"recipe": f"x,y~U[0,300], z~U[1.1,6], N={N}", "seed": seed})


def divergence_config(seed: int = 0, N: int = 500) -> Config:
    """500 blobs with the config-0 density (box 60*sqrt(N/1000))."""
    box = 60.0 * math.sqrt(N / 1000.0)
    return Config("DIV", uniform_slab(N, box, 1.1, 6.0, seed),
                  meta={"recipe": f"x,y~U[0,{box:g}], z~U[1.1,6], N={N}", "seed": seed})


# ---------------------------------------------------------------- rigid bodies

def _rot_z(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_quat(qv: np.ndarray) -> np.ndarray:
    """Rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = qv
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def boomerang_frame(spacing: float = 2.1) -> np.ndarray:
    """15 blobs in the body frame: corner at the origin, arms along +x and +y.

    Blob 0 is the shared corner (the tracking "cross point"); blobs 1..7 run
    along x and 8..14 along y, at the given centre spacing.
    """
    pts = [(0.0, 0.0, 0.0)]
    pts += [(spacing * m, 0.0, 0.0) for m in range(1, 8)]
    pts += [(0.0, spacing * m, 0.0) for m in range(1, 8)]
    return np.array(pts)


def icosahedron_frame() -> np.ndarray:
    """12 icosahedron vertices (0, +-1, +-phi) and cyclic permutations.

    Edge length is 2 (touching blobs of radius 1); circumradius sqrt(1+phi^2).
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-phi, phi):
            pts += [(0.0, s1, s2), (s1, s2, 0.0), (s2, 0.0, s1)]
    return np.array(pts)


def boomerang_suspension(n_bodies: int, box: float, zlo: float, zhi: float, seed: int,
                         spacing: float = 2.1) -> tuple[np.ndarray, np.ndarray]:
    """Boomerangs lying flat, each rotated uniformly about z.

    Cross points: x, y ~ U[0, box], z ~ U[zlo, zhi].  Returns positions
    (15 n_bodies, 3) and body offsets [n_bodies + 1].
    """
    rng = np.random.default_rng(seed)
    frame = boomerang_frame(spacing)
    pos = np.empty((n_bodies * 15, 3))
    for p in range(n_bodies):
        c = np.array([rng.uniform(0, box), rng.uniform(0, box), rng.uniform(zlo, zhi)])
        rot = _rot_z(rng.uniform(0.0, 2.0 * math.pi))
        pos[15 * p: 15 * (p + 1)] = c + frame @ rot.T
    offs = np.arange(0, 15 * n_bodies + 1, 15, dtype=np.int64)
    return pos, offs


def microroller_suspension(n_spheres: int, phi_area: float, seed: int,
                           zlo: float = 1.1, zhi: float = 4.0,
                           jitter: float = 1.1) -> tuple[np.ndarray, np.ndarray, float]:
    """12-blob spheres on a jittered square lattice at areal fraction phi_area.

    Sphere radius used for the packing fraction is R_v + a (vertex radius plus
    one blob radius).  The lowest point of each sphere's blob centres is at
    z_c - R_v ~ U[zlo, zhi].  Orientation: uniform random unit quaternion.
    Returns positions, body offsets and the box side.
    """
    rng = np.random.default_rng(seed)
    frame = icosahedron_frame()
    r_v = float(np.linalg.norm(frame[0]))
    r_p = r_v + 1.0
    side = int(math.ceil(math.sqrt(n_spheres)))
    box = math.sqrt(n_spheres * math.pi * r_p * r_p / phi_area)
    pitch = box / side
    pos = np.empty((n_spheres * 12, 3))
    for s in range(n_spheres):
        ix, iy = s % side, s // side
        cx = (ix + 0.5) * pitch + rng.uniform(-jitter, jitter)
        cy = (iy + 0.5) * pitch + rng.uniform(-jitter, jitter)
        cz = r_v + rng.uniform(zlo, zhi)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        pos[12 * s: 12 * (s + 1)] = np.array([cx, cy, cz]) + frame @ _rot_quat(q).T
    offs = np.arange(0, 12 * n_spheres + 1, 12, dtype=np.int64)
    return pos, offs, box


def config1(seed: int = 0) -> Config:
    """256 boomerangs (3840 blobs), spacing 2.1a, box 80, cross-point z in [1.5, 4]."""
    pos, offs = boomerang_suspension(256, 80.0, 1.5, 4.0, seed)
    return Config("C1", pos, body_offsets=offs,
                  meta={"recipe": "256 boomerangs, spacing 2.1, x,y~U[0,80], z~U[1.5,4], theta~U[0,2pi)",
                        "seed": seed})


def paperlike_boomerangs(n_bodies: int, seed: int = 0, spacing: float = 0.926,
                         density: float = 256.0 / 139.8 ** 2, zlo: float = 1.5,
                         zhi: float = 4.0, min_gap: float = 2.0,
                         max_tries: int = 2_000_000) -> Config:
    """Boomerangs at the paper's blob spacing with no inter-body blob overlap.

    Random sequential addition in a square box at the given number density
    of bodies: a candidate body is rejected when any of its blobs comes
    closer than ``min_gap`` to a blob of an accepted body.  Accepted bodies
    are binned by corner position in cells wider than two arm lengths plus
    the gap, so only the 3 x 3 neighbouring cells are checked.
    """
    rng = np.random.default_rng(seed)
    box = math.sqrt(n_bodies / density)
    frame = boomerang_frame(spacing)
    reach = 2.0 * float(np.linalg.norm(frame, axis=1).max()) + min_gap
    cells: dict[tuple[int, int], list[np.ndarray]] = {}
    bodies: list[np.ndarray] = []
    tries = 0
    while len(bodies) < n_bodies:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not place all bodies")
        c = np.array([rng.uniform(0, box), rng.uniform(0, box), rng.uniform(zlo, zhi)])
        cand = c + frame @ _rot_z(rng.uniform(0.0, 2.0 * math.pi)).T
        cx, cy = int(c[0] // reach), int(c[1] // reach)
        near = [b for dx in (-1, 0, 1) for dy in (-1, 0, 1) for b in cells.get((cx + dx, cy + dy), [])]
        if near:
            allp = np.concatenate(near)
            d2 = ((cand[:, None, :] - allp[None, :, :]) ** 2).sum(-1)
            if d2.min() < min_gap * min_gap:
                continue
        bodies.append(cand)
        cells.setdefault((cx, cy), []).append(cand)
    pos = np.concatenate(bodies)
    offs = np.arange(0, 15 * n_bodies + 1, 15, dtype=np.int64)
    return Config(f"PB{n_bodies}", pos, body_offsets=offs,
                  meta={"recipe": f"{n_bodies} boomerangs, spacing {spacing}, RSA gap {min_gap}, box {box:.2f}",
                        "seed": seed})


def config2(seed: int = 0, n_spheres: int = 16384) -> Config:
    """16384 twelve-blob microrollers (196608 blobs) at areal fraction 0.4."""
    pos, offs, box = microroller_suspension(n_spheres, 0.4, seed)
    return Config("C2", pos, body_offsets=offs,
                  meta={"recipe": f"{n_spheres} icosahedral 12-blob spheres, phi=0.4, box {box:.1f}, "
                                  "z_c-R_v~U[1.1,4], random SO(3)", "seed": seed})


def config3(seed: int = 0, n_systems: int = 64, lo: int = 500, hi: int = 20000) -> Config:
    """64 independent suspensions, blob counts log-uniform in [lo, hi].

    Each system is a boomerang (15-blob) or microroller (12-blob) suspension,
    chosen by a seeded coin flip; counts are rounded to whole bodies.
    """
    rng = np.random.default_rng(seed)
    parts, sys_offs, kinds = [], [0], []
    for s in range(n_systems):
        n_target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() < 0.5:
            nb = max(1, int(round(n_target / 15)))
            pos, _ = boomerang_suspension(nb, 80.0 * math.sqrt(nb / 256.0), 1.5, 4.0, sub_seed)
            kinds.append("boomerang")
        else:
            nb = max(1, int(round(n_target / 12)))
            pos, _, _ = microroller_suspension(nb, 0.4, sub_seed)
            kinds.append("sphere")
        parts.append(pos)
        sys_offs.append(sys_offs[-1] + pos.shape[0])
    return Config("C3", np.concatenate(parts), sys_offsets=np.array(sys_offs, dtype=np.int64),
                  meta={"recipe": "64 systems, N_s log-uniform [500,20000], boomerang or sphere",
                        "kinds": kinds, "seed": seed})
