"""Batched independent suspensions in one persistent launch (P13: systems
never interact) against per-system products and the oracle."""
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


@pytest.mark.parametrize("prec,k", [(0, 3), (0, 16), (1, 3), (1, 6), (1, 9), (1, 16)])
def test_small_systems_against_oracle(rp, orc, prec, k):
    """Overlapping systems (same region of space) must not interact.  FP32C
    with 6, 9 and 16 right-hand sides and FP64 with 16 take the matrix-core
    kernel (blocks of 8 and 16, work items of 64 targets), the others the
    vector kernel."""
    rng = np.random.default_rng(3)
    sizes = [1, 7, 300, 256, 513, 40, 65]
    parts = [np.column_stack([rng.uniform(0, 20, n), rng.uniform(0, 20, n), rng.uniform(0.5, 5, n)]) for n in sizes]
    pos = np.concatenate(parts)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    F = wl.gaussian((k, pos.shape[0], 3), 4)
    U = rp.matvec_batched(_t(pos), offs, _t(F), precision=prec).cpu().numpy()
    for s in range(len(sizes)):
        sl = slice(offs[s], offs[s + 1])
        for l in range(k):
            ref = orc.matvec(pos[sl], F[l, sl])
            check(U[l, sl], ref, 1e-12 if prec == 0 else 1e-5, f"batched prec={prec} system={s} rhs={l}")


def test_config3_against_per_system_launches(rp, orc):
    """64 suspensions, 500-20000 blobs, 16 RHS, FP32C: the persistent launch
    equals the per-system multi-RHS products to FP32C accuracy, and sampled
    rows match the FP64 oracle."""
    cfg = wl.config3(seed=0)
    offs = cfg.sys_offsets
    k = 16
    F = wl.gaussian((k, cfg.N, 3), 5)
    pos, Ft = _t(cfg.pos), _t(F)
    U = rp.matvec_batched(pos, offs, Ft, precision=1)
    worst = (0.0, 0.0)
    for s in range(len(offs) - 1):
        sl = slice(int(offs[s]), int(offs[s + 1]))
        Us = rp.matvec_multi(pos[sl].contiguous(), Ft[:, sl].contiguous(), precision=1)
        r, e = check(U[:, sl].cpu().numpy(), Us.cpu().numpy(), 2e-6, f"C3 system {s} batched vs per-system")
        worst = (max(worst[0], r), max(worst[1], e))
    print(f"C3 batched vs per-system worst rel={worst[0]:.3e} entry={worst[1]:.3e} (N_tot={cfg.N})", flush=True)
    Uc = U.cpu().numpy()
    rng = np.random.default_rng(1)
    for s in sorted(set(rng.choice(len(offs) - 1, 4, replace=False)) | {0, len(offs) - 2}):
        b0, b1 = int(offs[s]), int(offs[s + 1])
        rows = np.concatenate([rng.choice(b1 - b0, 16, replace=False), [0, b1 - b0 - 1]])
        for l in (0, 7, 15):
            ref = orc.matvec(cfg.pos[b0:b1], F[l, b0:b1], rows=rows)
            check(Uc[l, b0:b1][rows], ref, 1e-5, f"C3 system {s} rhs {l} sampled rows vs oracle")
