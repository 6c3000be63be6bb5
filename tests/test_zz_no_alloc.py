"""The product entry point that allocates nothing (rpy_wall_matvec_noalloc,
its workspace a fixed device array in the library) against the ordinary
entry point rpy_wall_matvec, through the C ABI: two calls in a row, the
second on a smaller input, in both precisions.  Same kernels and launch
shapes, so the results are the same bits; the FP64 oracle bars (1e-12 FP64,
1e-5 FP32C, per entry too) are asserted as well."""
import ctypes

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


def _call(rp, fn, pos, f, prec, ws=None):
    lib = rp.lib()
    out = torch.full_like(f, float("nan"))
    st = torch.cuda.current_stream().cuda_stream
    N = pos.shape[0]
    if fn == "noalloc":
        rc = lib.rpy_wall_matvec_noalloc(pos.data_ptr(), f.data_ptr(), out.data_ptr(), N, 0.9, 1.3, prec, st)
    else:
        rc = lib.rpy_wall_matvec(pos.data_ptr(), f.data_ptr(), out.data_ptr(), N, 0.9, 1.3, prec, ws.data_ptr(),
                                 ws.numel(), st)
    assert rc == rp.OK, rc
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_matvec_two_calls(rp, orc, prec):
    tol = 1e-12 if prec == 0 else 1e-5
    for N, seed in ((3840, 1), (777, 2)):  # the second call smaller than the first
        rng = np.random.default_rng(seed)
        box = 2.0 * np.sqrt(N)
        pos = np.column_stack([rng.uniform(0, box, N), rng.uniform(0, box, N), rng.uniform(0.3, 4.0, N)]) * 0.9
        pos[2] = pos[1]
        f = rng.standard_normal((N, 3))
        tp, tf = _t(pos), _t(f)
        ws = torch.empty(rp.workspace_bytes(rp.OP_MATVEC, N, 1, precision=prec), dtype=torch.uint8, device="cuda")
        ref_gpu = _call(rp, "matvec", tp, tf, prec, ws)
        got = _call(rp, "noalloc", tp, tf, prec)
        print(f"noalloc N={N} prec={prec} identical={np.array_equal(got, ref_gpu)}", flush=True)
        assert np.array_equal(got, ref_gpu)
        check(got, orc.matvec(pos, f, 0.9, 1.3), tol, f"noalloc N={N} prec={prec} vs oracle")


def test_noalloc_refuses_oversized_problem(rp):
    pos = _t(np.ones((20000, 3)))
    out = torch.empty_like(pos)
    lib = rp.lib()
    assert lib.rpy_wall_matvec_noalloc(pos.data_ptr(), pos.data_ptr(), out.data_ptr(), 20000, 1.0, 1.0, 0,
                                       None) == rp.ENOMEM
    # the binding reports it as an error
    with pytest.raises(rp.RpywError):
        rp.matvec_noalloc(pos, pos)
