"""GPU preconditioned Lanczos (Sec. II.B) against the oracle's Lanczos and
dense square roots.  Small cases run both drivers: the fused one (four
launches per step, used whenever the product goes through the symmetric
kernel) and the unfused one."""

import numpy as np
import pytest

from paper_1709_02410_amd import workloads as wl
from parity_util import check, krylov_path

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_02410_amd import rpywall
    rpywall.lib()
    return rpywall


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_path = krylov_path


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("bodies", [True, False])
def test_small_against_dense_root(rp, orc, bodies, fused):
    pos, offs = wl.boomerang_suspension(12, 25.0, 1.5, 4.0, seed=3)
    offs = offs if bodies else None
    W = wl.gaussian(pos.shape, 4)
    ref = orc.dense_sqrt(pos, W, offs)
    with _path(rp, len(pos), fused):
        out, it, err, ok = rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-10)
    got = out.cpu().numpy()
    print(f"dense-root bodies={bodies} iters={it}", flush=True)
    assert ok
    check(got, ref, 1e-9, f"lanczos vs dense root bodies={bodies}")


def test_boomerangs_3840_tol_1e6(rp, orc):
    """256 boomerangs (3840 blobs), FP64 products, tolerance 1e-6: same
    iteration count and iterate as the oracle's Lanczos, and within 10 tol
    of the converged root (oracle at 1e-12)."""
    cfg = wl.config1(seed=0)
    W = wl.gaussian(cfg.pos.shape, 1)
    out, it, err, ok = rp.lanczos_sqrt(_t(cfg.pos), _t(W), body_offsets=cfg.body_offsets, tol=1e-6)
    got = out.cpu().numpy()
    ref6, it6, _, ok6 = orc.lanczos_sqrt(cfg.pos, W, cfg.body_offsets, tol=1e-6)
    ref12, it12, _, _ = orc.lanczos_sqrt(cfg.pos, W, cfg.body_offsets, tol=1e-12)
    print(f"C1 iters gpu={it} oracle={it6} (tol 1e-12: {it12}) rel-same-tol={_rel(got, ref6):.3e} "
          f"rel-converged={_rel(got, ref12):.3e}", flush=True)
    assert ok and ok6 and it == it6
    check(got, ref6, 1e-9, "C1 lanczos vs oracle lanczos, same tolerance")
    # Truncation error of the tolerance-1e-6 iterate (not a parity figure):
    # the stopping rule bounds the relative L2 change of the iterate, so the
    # entry bound is the L2 bound carried to one entry, |e|_inf <= |e|_2.
    ref_scale = float(np.linalg.norm(ref12) / np.abs(ref12).max())
    check(got, ref12, 1e-5, "C1 lanczos vs converged oracle root", elem_bar=1e-5 * ref_scale)


def test_per_blob_preconditioner_config0(rp, orc):
    cfg = wl.config0(seed=1)
    W = wl.gaussian(cfg.pos.shape, 2)
    out, it, err, ok = rp.lanczos_sqrt(_t(cfg.pos), _t(W), tol=1e-8)
    ref, it_o, _, _ = orc.lanczos_sqrt(cfg.pos, W, None, tol=1e-8)
    assert ok and abs(it - it_o) <= 1
    check(out.cpu().numpy(), ref, 1e-7, "C0 per-blob preconditioner lanczos")


@pytest.mark.parametrize("fused", [False, True])
def test_not_converged_returns_best_iterate(rp, orc, fused):
    pos, offs = wl.boomerang_suspension(8, 20.0, 1.5, 4.0, seed=5)
    W = wl.gaussian(pos.shape, 6)
    with _path(rp, len(pos), fused):
        out, it, err, ok = rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-14, max_iter=3)
        ref, it_o, _, ok_o = orc.lanczos_sqrt(pos, W, offs, tol=1e-14, max_iter=3)
        assert not ok and not ok_o and it == 3 and it_o == 3
        check(out.cpu().numpy(), ref, 1e-12, f"lanczos best iterate after max_iter fused={fused}")
        with pytest.raises(rp.RpywError):
            rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-14, max_iter=3, strict=True)


@pytest.mark.parametrize("fused", [False, True])
def test_non_spd_block_is_reported(rp, fused):
    """A body with a blob on the wall (B = 0) has a singular block."""
    pos, offs = wl.boomerang_suspension(2, 10.0, 1.5, 2.0, seed=7)
    pos[3, 2] = 0.0
    W = wl.gaussian(pos.shape, 1)
    with _path(rp, len(pos), fused), pytest.raises(rp.RpywError) as ei:
        rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-6)
    assert ei.value.status == rp.ENOTSPD


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("N,bodies", [(1, False), (2, False), (15, True)])
def test_exhausted_krylov_space(rp, orc, N, bodies, fused):
    """Tiny problems whose Krylov space is exhausted within a few steps (3N
    at most; one body with the block preconditioner: the preconditioned
    operator is the identity, one step): beta reaches zero, which the
    iteration must detect as convergence and return the exact root."""
    rng = np.random.default_rng(N)
    if bodies:
        pos = wl.boomerang_frame(2.1) + np.array([5.0, 5.0, 3.0])
        offs = np.array([0, 15], dtype=np.int64)
    else:
        pos = np.column_stack([rng.uniform(0, 4, N), rng.uniform(0, 4, N), rng.uniform(1.5, 3.0, N)])
        offs = None
    W = wl.gaussian(pos.shape, 9)
    ref = orc.dense_sqrt(pos, W, offs)
    with _path(rp, len(pos), fused):
        out, it, err, ok = rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-12, max_iter=3 * len(pos) + 4)
    got = out.cpu().numpy()
    print(f"exhausted N={len(pos)} bodies={bodies} iters={it}", flush=True)
    assert ok and it <= 3 * len(pos)
    check(got, ref, 1e-11, f"exhausted Krylov space N={len(pos)}")


@pytest.mark.parametrize("fused", [False, True])
def test_zero_vector(rp, fused):
    pos, offs = wl.boomerang_suspension(2, 10.0, 1.5, 2.0, seed=7)
    with _path(rp, len(pos), fused):
        out, it, err, ok = rp.lanczos_sqrt(_t(pos), _t(np.zeros_like(pos)), body_offsets=offs)
    assert ok and it == 0 and float(out.abs().max()) == 0.0


def test_microrollers_fp32_products(rp):
    """196608-blob microroller suspension (12-blob bodies): Lanczos with
    FP32C products and FP64 Krylov arithmetic against the all-FP64 run."""
    cfg = wl.config2(seed=0)
    W = wl.gaussian(cfg.pos.shape, 3)
    pos, w = _t(cfg.pos), _t(W)
    o64, it64, _, ok64 = rp.lanczos_sqrt(pos, w, body_offsets=cfg.body_offsets, tol=1e-6, precision=0)
    o32, it32, _, ok32 = rp.lanczos_sqrt(pos, w, body_offsets=cfg.body_offsets, tol=1e-6, precision=1)
    print(f"C2 lanczos iters fp64={it64} fp32c={it32}", flush=True)
    assert ok64 and ok32 and abs(it64 - it32) <= 1
    check(o32.cpu().numpy(), o64.cpu().numpy(), 1e-5, "C2 lanczos fp32c vs fp64")


def test_iterations_independent_of_size(rp):
    """Sec. II.B / IV.B: preconditioned iterations at tolerance 1e-3 stay
    about 5 and do not grow with the number of boomerangs."""
    its = []
    for nb in (64, 256, 1024):
        cfg = wl.paperlike_boomerangs(nb, seed=2)
        W = wl.gaussian(cfg.pos.shape, 9)
        _, it, _, ok = rp.lanczos_sqrt(_t(cfg.pos), _t(W), body_offsets=cfg.body_offsets, tol=1e-3)
        _, it_u, _, _ = rp.lanczos_sqrt(_t(cfg.pos), _t(W), tol=1e-3)
        its.append((it, it_u))
        assert ok
    print(f"iterations (pc, per-blob) by size: {its}", flush=True)
    pc = [p for p, _ in its]
    assert max(pc) <= 8 and max(pc) - min(pc) <= 1


@pytest.mark.parametrize("fused", [False, True])
def test_largest_bodies_42_blobs(rp, orc, fused):
    """Bodies of the largest supported size (42 blobs, a 6 x 7 plate; the
    preconditioner factors need 129 KB of LDS) next to small ones: the
    Lanczos root and the rigid solve against the oracle."""
    gx, gy = np.meshgrid(np.arange(6) * 1.9, np.arange(7) * 1.9)
    plate = np.column_stack([gx.ravel(), gy.ravel(), np.full(42, 3.0)])
    pos = np.concatenate([plate, plate + [16.0, 0.0, 0.5], plate[[0, 1, 6, 7, 13]] + [0.0, 16.0, 0.0]])
    offs = np.array([0, 42, 84, 89])
    W = wl.gaussian(pos.shape, 21)
    with _path(rp, len(pos), fused):
        out, it, err, ok = rp.lanczos_sqrt(_t(pos), _t(W), body_offsets=offs, tol=1e-10)
    ref = orc.dense_sqrt(pos, W, offs)
    assert ok
    check(out.cpu().numpy(), ref, 1e-8, "42-blob bodies lanczos")
    q = np.array([pos[offs[p]:offs[p + 1]].mean(0) for p in range(3)])
    FT = wl.gaussian((3, 6), 22)
    lam_ref, U_ref = orc.rigid_solve(pos, q, offs, None, FT)
    lam, U, it, res, ok = rp.rigid_solve(_t(pos), _t(q), offs, None, _t(FT), tol=1e-11)
    assert ok
    check(U.cpu().numpy(), U_ref, 1e-8, "42-blob bodies rigid U")


@pytest.mark.parametrize("fused", [False, True])
def test_back_to_back_calls_and_two_streams(rp, orc, fused):
    """The solvers return with their last kernels (and up to two speculative
    steps) still queued, and their pinned scalar slots are shared between
    calls: several Lanczos roots and rigid solves issued back to back, on one
    stream and on two streams, without synchronising in between, equal the
    same calls made one at a time."""
    with _path(rp, 180, fused):
        _back_to_back(rp)


def _back_to_back(rp):
    pos, offs = wl.boomerang_suspension(12, 25.0, 1.5, 4.0, seed=8)
    Ws = [wl.gaussian(pos.shape, 40 + i) for i in range(4)]
    q = pos[offs[:-1]].copy()
    FT = wl.gaussian((len(offs) - 1, 6), 50)
    p = _t(pos)
    ref = []
    for W in Ws:
        out, _, _, ok = rp.lanczos_sqrt(p, _t(W), body_offsets=offs, tol=1e-10)
        torch.cuda.synchronize()
        ref.append(out.cpu().numpy())
    lam_r, U_r, _, _, _ = rp.rigid_solve(p, _t(q), offs, _t(Ws[0]), _t(FT), tol=1e-10)
    torch.cuda.synchronize()
    U_r = U_r.cpu().numpy()
    # back to back on the current stream
    outs = [rp.lanczos_sqrt(p, _t(W), body_offsets=offs, tol=1e-10)[0] for W in Ws]
    U1 = rp.rigid_solve(p, _t(q), offs, _t(Ws[0]), _t(FT), tol=1e-10)[1]
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r)
    assert np.array_equal(U1.cpu().numpy(), U_r)
    # alternating between two streams (default priority)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for i, W in enumerate(Ws):
        with torch.cuda.stream(s1 if i % 2 == 0 else s2):
            Wt = _t(W)
            outs.append(rp.lanczos_sqrt(p, Wt, body_offsets=offs, tol=1e-10)[0])
    with torch.cuda.stream(s2):
        U2 = rp.rigid_solve(p, _t(q), offs, _t(Ws[0]), _t(FT), tol=1e-10)[1]
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert np.array_equal(o.cpu().numpy(), r)
    assert np.array_equal(U2.cpu().numpy(), U_r)
