"""GPU pseudo-periodic mobility (Sec. IV.B suspensions: minimum image plus the
8 periodic images along the wall) against the oracle: products, the
preconditioned Lanczos root and the rigid solve."""
import math

import numpy as np
import pytest

from paper_1709_02410_amd import workloads as wl
from parity_util import check

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def rp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_02410_amd import rpywall
    rpywall.lib()
    return rpywall


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _cell(N, seed, a=1.0):
    """Blobs in a cell of side about 2 sqrt(N) a (at least 6a), some outside
    it (wrapped by the library), some below z = a, one overlapping pair."""
    rng = np.random.default_rng(seed)
    L = max(6.0, 2.0 * math.sqrt(N)) * a
    Ly = 1.3 * L
    pos = np.column_stack([rng.uniform(0, L, N), rng.uniform(0, Ly, N), rng.uniform(0.3, 4.0, N) * a])
    pos[::5, 0] += L * rng.integers(-2, 3, len(pos[::5]))
    if N >= 3:
        pos[2] = pos[1] + np.array([0.4, -0.2, 0.1]) * a
    return pos, (L, Ly)


@pytest.mark.parametrize("N", [1, 7, 300, 777, 2100])
@pytest.mark.parametrize("prec", [0, 1])
def test_periodic_product_matches_oracle(rp, orc, N, prec):
    a, eta = 0.9, 1.2
    pos, box = _cell(N, 100 + N, a)
    f = wl.gaussian(pos.shape, 200 + N)
    ref = orc.matvec(pos, f, a, eta, box=box)
    for sym, ipw in ((1, 1), (1, 2), (2, 1), (2, 3), (0, 2)):  # groups of 256, of 64, of 64
        rp.set_shape(prec, N, 1, tpl=1, tile=256, kblk=1, sym=sym, ipw=ipw)
        got = rp.matvec(_t(pos), _t(f), a, eta, precision=prec, box=box).cpu().numpy()
        check(got, ref, TOL[prec], f"periodic N={N} prec={prec} sym={sym} ipw={ipw}")
    rp.reset_shape(prec, N, 1)


@pytest.mark.parametrize("prec", [0, 1])
def test_periodic_4096_boomerangs_sampled_rows(rp, orc, prec):
    """The benchmark's large periodic workload: 4096 paper-like boomerangs
    (61440 blobs) in their cell (side 559.2 a), in the launch shape the
    benchmark times (the default: symmetric kernel over groups of 256,
    unsegmented); 96 sampled rows plus the first and the ragged last blob
    against the oracle's explicit image sum."""
    cfg = wl.paperlike_boomerangs(4096, seed=2)
    Lc = 139.8 * math.sqrt(4096 / 256.0)
    f = wl.gaussian(cfg.pos.shape, 12)
    sh = rp.get_shape(prec, cfg.N, 1)
    print(f"periodic 61440 shape prec={prec}: {sh}", flush=True)
    assert sh["sym"] == 1
    got = rp.matvec(_t(cfg.pos), _t(f), precision=prec, box=(Lc, Lc)).cpu().numpy()
    rows = np.concatenate([np.random.default_rng(13).choice(cfg.N, 96, replace=False), [0, cfg.N - 1]])
    ref = orc.matvec(cfg.pos, f, rows=rows, box=(Lc, Lc))
    check(got[rows], ref, TOL[prec], f"periodic 61440 prec={prec} sampled rows")


@pytest.mark.parametrize("prec", [0, 1])
def test_paper_suspension_cell(rp, orc, prec):
    """256 boomerangs with the paper's geometry in their periodic cell
    (3840 blobs, cell 139.8 a): three right-hand sides at once."""
    cfg = wl.paperlike_boomerangs(256, seed=2)
    L = 139.8
    F = wl.gaussian((3, cfg.N, 3), 7)
    U = rp.matvec_periodic(_t(cfg.pos), _t(F), (L, L), precision=prec).cpu().numpy()
    for l in range(3):
        ref = orc.matvec(cfg.pos, F[l], box=(L, L))
        check(U[l], ref, TOL[prec], f"paper cell prec={prec} rhs={l}")


def test_wrapping_and_large_cell(rp):
    """Positions shifted by whole cells give the same velocities; a huge
    cell reproduces the open-domain product."""
    pos, box = _cell(500, 9)
    f = _t(wl.gaussian(pos.shape, 10))
    u = rp.matvec(_t(pos), f, box=box)
    moved = pos + np.array([3 * box[0], -2 * box[1], 0.0])
    assert float((rp.matvec(_t(moved), f, box=box) - u).norm() / u.norm()) <= 1e-13
    # (blobs inside [0, 1e7): wrapping far-outside positions into a cell
    # that large would itself cost precision, ulp(1e7) ~ 2e-9)
    inside = pos.copy()
    inside[:, 0] = np.mod(inside[:, 0], box[0])
    u_open = rp.matvec(_t(inside), f)
    u_big = rp.matvec(_t(inside), f, box=(1e7, 1.1e7))
    assert float((u_big - u_open).norm() / u_open.norm()) <= 1e-12


def test_periodic_lanczos_matches_dense_root(rp, orc):
    cfg = wl.paperlike_boomerangs(12, seed=5)
    L = math.sqrt(12 / (256.0 / 139.8 ** 2))
    W = wl.gaussian(cfg.pos.shape, 11)
    ref = orc.dense_sqrt(cfg.pos, W, cfg.body_offsets, box=(L, L))
    out, it, err, ok = rp.lanczos_sqrt(_t(cfg.pos), _t(W), body_offsets=cfg.body_offsets, tol=1e-10, box=(L, L))
    print(f"periodic lanczos iters={it}", flush=True)
    assert ok
    check(out.cpu().numpy(), ref, 1e-8, "periodic lanczos vs dense root")


def test_periodic_rigid_solve_matches_dense(rp, orc):
    cfg = wl.paperlike_boomerangs(12, seed=6)
    L = math.sqrt(12 / (256.0 / 139.8 ** 2))
    offs = cfg.body_offsets
    q = cfg.pos[offs[:-1]].copy()
    FT = wl.gaussian((len(offs) - 1, 6), 12)
    slip = wl.gaussian(cfg.pos.shape, 13)
    lam_ref, U_ref = orc.rigid_solve(cfg.pos, q, offs, slip, FT, box=(L, L))
    lam, U, it, res, ok = rp.rigid_solve(_t(cfg.pos), _t(q), offs, _t(slip), _t(FT), tol=1e-11, box=(L, L))
    print(f"periodic rigid iters={it}", flush=True)
    assert ok
    check(U.cpu().numpy(), U_ref, 1e-8, "periodic rigid U")
    check(lam.cpu().numpy(), lam_ref, 1e-7, "periodic rigid lambda")


@pytest.mark.parametrize("prec", [0, 1])
def test_small_cell_images_overlap(rp, orc, prec):
    """Cells narrower than 4.5 a, where periodic images other than the minimum
    one overlap their targets (r < 2 a): the kernel keeps the overlap branch
    for every image there (the wider-cell FP64 path skips it for the eight
    shifted images)."""
    rng = np.random.default_rng(77)
    N, box = 30, (4.0, 4.2)
    pos = np.column_stack([rng.uniform(0, box[0], N), rng.uniform(0, box[1], N), rng.uniform(0.8, 3.0, N)])
    f = wl.gaussian(pos.shape, 78)
    ref = orc.matvec(pos, f, box=box)
    got = rp.matvec(_t(pos), _t(f), precision=prec, box=box).cpu().numpy()
    check(got, ref, TOL[prec], f"small cell prec={prec}")
    # just above the threshold: the shifted images are at least 2.25 a away
    box2 = (4.6, 4.7)
    ref2 = orc.matvec(pos, f, box=box2)
    got2 = rp.matvec(_t(pos), _t(f), precision=prec, box=box2).cpu().numpy()
    check(got2, ref2, TOL[prec], f"cell above threshold prec={prec}")
