"""GPU VJP and divergence against the oracle, central differences and the
random-finite-difference estimate of the drift (Sec. III)."""
import math

import numpy as np
import pytest

from paper_1709_02410_amd import workloads as wl
from parity_util import check

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


def _mixed(n, seed, box=None):
    rng = np.random.default_rng(seed)
    box = box or 2.0 * math.sqrt(n)
    return np.column_stack([rng.uniform(0, box, n), rng.uniform(0, box, n), rng.uniform(0.3, 4.0, n)])


# The derivative paths carry the product's precision targets: FP64 1e-12 and
# FP32C 1e-5 relative L2 against the FP64 oracle, and the same per entry
# against the largest reference entry.
DTOL = {0: 1e-12, 1: 1e-5}


@pytest.mark.parametrize("prec", [0, 1])
def test_vjp_matches_oracle(rp, orc, prec):
    """Blobs below z = a, overlapping pairs, ragged size (several tiles)."""
    a, eta = 0.8, 1.1
    pos = _mixed(777, 1) * a
    f = wl.gaussian(pos.shape, 2)
    g = wl.gaussian(pos.shape, 3)
    gp_ref, gf_ref = orc.vjp(pos, f, g, a, eta)
    gp, gf = rp.matvec_vjp(_t(pos), _t(f), _t(g), a, eta, precision=prec)
    check(gp.cpu().numpy(), gp_ref, DTOL[prec], f"vjp 777 prec={prec} grad_pos")
    check(gf.cpu().numpy(), gf_ref, DTOL[prec], f"vjp 777 prec={prec} grad_f")


@pytest.mark.parametrize("prec", [0, 1])
def test_vjp_50k_sampled_rows_match_oracle(rp, orc, prec):
    """The differentiation workload (5e4 blobs, box 300) in the launch shape
    the benchmark times (the default: symmetric kernel over groups of 256,
    unsegmented): both gradients on 128 sampled blobs against the oracle's
    dual-number VJP of those rows."""
    cfg = wl.config4(seed=0)
    f = wl.gaussian(cfg.pos.shape, 1)
    g = wl.gaussian(cfg.pos.shape, 2)
    sh = rp.get_shape(prec, cfg.N, 1)
    print(f"C4 vjp shape prec={prec}: {sh}", flush=True)
    assert sh["sym"] == 1  # groups of 256 at this size
    gp, gf = rp.matvec_vjp(_t(cfg.pos), _t(f), _t(g), precision=prec)
    gp, gf = gp.cpu().numpy(), gf.cpu().numpy()
    rows = np.random.default_rng(8).choice(cfg.N, 128, replace=False)
    rows = np.concatenate([rows, [0, cfg.N - 1]])  # first group and the ragged last one
    gp_ref, gf_ref = orc.vjp(cfg.pos, f, g, rows=rows)
    check(gp[rows], gp_ref, DTOL[prec], f"C4 vjp prec={prec} grad_pos sampled rows")
    check(gf[rows], gf_ref, DTOL[prec], f"C4 vjp prec={prec} grad_f sampled rows")


@pytest.mark.parametrize("prec", [0, 1])
def test_vjp_central_differences_50k(rp, prec):
    """Differentiation workload (5e4 blobs, box 300): VJP against central
    differences (h = 1e-4) of the FP64 GPU product, on 8 random directions
    and 64 sampled coordinates."""
    cfg = wl.config4(seed=0)
    pos = _t(cfg.pos)
    f = _t(wl.gaussian(cfg.pos.shape, 1))
    g = _t(wl.gaussian(cfg.pos.shape, 2))
    gp, gf = rp.matvec_vjp(pos, f, g, precision=prec)
    h = 1e-4

    def L(p):
        return float((g * rp.matvec(p, f, precision=0)).sum())

    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(8):
        d = _t(rng.standard_normal(cfg.pos.shape))
        fd = (L(pos + h * d) - L(pos - h * d)) / (2 * h)
        an = float((gp * d).sum())
        worst = max(worst, abs(fd - an) / abs(fd))
    gmax = float(gp.abs().max())
    worst_c = 0.0
    for flat in rng.choice(cfg.N * 3, 64, replace=False):
        e = torch.zeros_like(pos).view(-1)
        e[flat] = h
        e = e.view(-1, 3)
        fd = (L(pos + e) - L(pos - e)) / (2 * h)
        worst_c = max(worst_c, abs(fd - float(gp.view(-1)[flat])) / gmax)
    print(f"vjp-fd prec={prec} directional rel={worst:.3e} coordinate rel={worst_c:.3e}", flush=True)
    assert worst <= 1e-4 and worst_c <= 1e-4
    gf_ref = rp.matvec(pos, g, precision=prec)
    check(gf.cpu().numpy(), gf_ref.cpu().numpy(), 1e-14 if prec == 0 else 1e-6, f"C4 grad_f vs product prec={prec}")


def test_autograd_function(rp):
    pos = _t(_mixed(300, 4)).requires_grad_(True)
    f = _t(wl.gaussian((300, 3), 5)).requires_grad_(True)
    g = _t(wl.gaussian((300, 3), 6))
    u = rp.rpy_wall_matvec(pos, f)
    (u * g).sum().backward()
    gp, gf = rp.matvec_vjp(pos.detach(), f.detach(), g)
    assert torch.equal(pos.grad, gp) and torch.equal(f.grad, gf)


@pytest.mark.parametrize("prec", [0, 1])
def test_divergence_matches_oracle(rp, orc, prec):
    cfg = wl.divergence_config(seed=0)
    pos = cfg.pos.copy()
    pos[:40, 2] = np.linspace(0.2, 0.99, 40)  # some blobs overlap the wall
    ref = orc.divergence(pos)
    got = rp.divergence(_t(pos), precision=prec).cpu().numpy()
    check(got, ref, DTOL[prec], f"divergence 500 prec={prec}")


@pytest.mark.parametrize("N", [1, 37, 64, 130])
def test_divergence_small_and_ragged_sizes(rp, orc, N):
    """One wave per target with the sources dealt over the 64 lanes: fewer
    sources than lanes, exactly one per lane, and a ragged second round."""
    rng = np.random.default_rng(N)
    pos = np.column_stack([rng.uniform(0, 12, N), rng.uniform(0, 12, N), rng.uniform(0.3, 4.0, N)])
    if N > 2:
        pos[2] = pos[1] + [0.4, 0.2, 0.1]  # an overlapping pair
    ref = orc.divergence(pos)
    got = rp.divergence(_t(pos), precision=0).cpu().numpy()
    check(got, ref, DTOL[0], f"divergence N={N}")


@pytest.mark.parametrize("prec,delta", [(0, 1e-6), (1, 1e-3)])
def test_rfd_drift_estimate_matches_exact_divergence(rp, prec, delta):
    """Centred RFD with Delta P = Delta Q = W (Sec. III) on the 500-blob
    workload: 1e4 samples, all 2e4 displaced systems in one batched launch;
    per-component z-scores and a global chi-square against the exact
    divergence."""
    cfg = wl.divergence_config(seed=0)
    N = cfg.N
    S = 10_000
    div = rp.divergence(_t(cfg.pos), precision=0).cpu().numpy()
    rng = np.random.default_rng(17)
    W = rng.standard_normal((S, N, 3))
    pos = np.concatenate([cfg.pos[None] + 0.5 * delta * W, cfg.pos[None] - 0.5 * delta * W], 0).reshape(-1, 3)
    F = np.concatenate([W, W], 0).reshape(1, -1, 3)
    offs = np.arange(0, 2 * S * N + 1, N, dtype=np.int64)
    U = rp.matvec_batched(_t(pos), offs, _t(F), precision=prec).cpu().numpy().reshape(2, S, N, 3)
    samples = (U[0] - U[1]) / delta
    mean = samples.mean(0)
    se = samples.std(0, ddof=1) / math.sqrt(S)
    z = (mean - div) / se
    chi2 = float((z ** 2).sum())
    dof = z.size
    print(f"rfd prec={prec} max|z|={np.abs(z).max():.2f} chi2/dof={chi2 / dof:.3f}", flush=True)
    assert np.abs(z).max() < 5.0
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


@pytest.mark.parametrize("N", [1, 7, 65, 300, 513, 1300])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sym", [1, 2])
def test_symmetric_vjp_matches_oracle(rp, orc, N, prec, sym):
    """The symmetric VJP kernel (one pair gradient per unordered pair, used
    for both blobs), over groups of 256 (sym 1) and of 64 blobs (sym 2),
    forced at small and ragged sizes, with blobs below the wall and
    overlapping pairs."""
    a, eta = 0.8, 1.1
    pos = _mixed(N, 10 + N) * a
    if N >= 3:
        pos[2] = pos[1] + np.array([0.3, 0.0, 0.1]) * a
    f = wl.gaussian(pos.shape, 20 + N)
    g = wl.gaussian(pos.shape, 30 + N)
    gp_ref, gf_ref = orc.vjp(pos, f, g, a, eta)
    for ipw in (1, 2):
        rp.set_shape(prec, N, 1, tpl=1, tile=256, kblk=1, sym=sym, ipw=ipw)
        gp, gf = rp.matvec_vjp(_t(pos), _t(f), _t(g), a, eta, precision=prec)
        what = f"sym vjp N={N} prec={prec} sym={sym} ipw={ipw}"
        check(gp.cpu().numpy(), gp_ref, DTOL[prec], what + " grad_pos")
        check(gf.cpu().numpy(), gf_ref, DTOL[prec], what + " grad_f")
    rp.reset_shape(prec, N, 1)
