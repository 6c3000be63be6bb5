"""Python binding of librpywall.so (the C ABI in include/rpywall.h).

Argument marshalling only: tensors are checked (float64, contiguous, on the
GPU), a workspace is taken from PyTorch's caching allocator, and the C entry
point is called on PyTorch's current HIP stream.  Every step of the
computation runs in the library's HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpywall.so")

FP64 = 0
FP32C = 1
OP_MATVEC, OP_BATCHED, OP_LANCZOS, OP_VJP, OP_DIVERGENCE, OP_RIGID, OP_TS = range(7)

OK, NOT_CONVERGED, EINVAL, EHIP, ENOMEM, ENOTSPD = 0, 1, -1, -2, -3, -4

_c_dp = ctypes.c_void_p
_lib = None


class RpywError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib().rpyw_strerror(status).decode()} (status {status})")


def lib():
    """Load librpywall.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1709_02410_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, dbl, sz, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "rpy_wall_matvec": [vp, vp, vp, i64, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_matvec_multi": [vp, vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_matvec_noalloc": [vp, vp, vp, i64, dbl, dbl, ctypes.c_int, vp],
        "rpy_wall_matvec_periodic": [vp, vp, vp, i64, i32, dbl, dbl, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_lanczos_sqrt_periodic": [vp, vp, vp, i64, dbl, dbl, dbl, dbl, i64p, i32, dbl, i32, ctypes.c_int,
                                           vp, sz, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp],
        "rpy_wall_rigid_solve_periodic": [vp, vp, i64p, i32, vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, dbl, i32,
                                          ctypes.c_int, vp, sz, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp],
        "rpy_wall_matvec_batched": [vp, i64p, i32, vp, vp, i32, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_lanczos_sqrt": [vp, vp, vp, i64, dbl, dbl, i64p, i32, dbl, i32, ctypes.c_int, vp, sz,
                                  ctypes.POINTER(i32), ctypes.POINTER(dbl), vp],
        "rpy_wall_rigid_solve": [vp, vp, i64p, i32, vp, vp, vp, vp, i64, dbl, dbl, dbl, i32, ctypes.c_int, vp, sz,
                                 ctypes.POINTER(i32), ctypes.POINTER(dbl), vp],
        "rpy_wall_body_blobs": [vp, vp, vp, i64p, i32, vp, i64, vp, sz, vp],
        "rpy_wall_body_move": [vp, vp, vp, dbl, i32, vp, vp, vp],
        "rpy_wall_ts_predict": [vp, vp, vp, i64p, i32, i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl, dbl, dbl, dbl,
                                i32, ctypes.c_int, vp, vp, vp, vp, sz, vp, sz, ctypes.POINTER(i32), vp],
        "rpy_wall_ts_correct": [vp, vp, vp, vp, vp, i64p, i32, i64, vp, vp, dbl, dbl, dbl, dbl, dbl, dbl, i32,
                                ctypes.c_int, vp, vp, vp, sz, ctypes.POINTER(i32), vp],
        "rpy_wall_emt_step": [vp, vp, vp, i64p, i32, i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl, dbl, dbl,
                              dbl, i32, ctypes.c_int, vp, vp, vp, sz, ctypes.POINTER(i32), vp],
        "rpy_wall_emrfd_step": [vp, vp, vp, i64p, i32, i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl, dbl, dbl,
                                dbl, i32, ctypes.c_int, vp, vp, vp, sz, ctypes.POINTER(i32), vp],
        "rpy_wall_matvec_vjp": [vp, vp, vp, vp, vp, i64, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_divergence": [vp, vp, i64, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpy_wall_autotune": [vp, vp, vp, i64, i32, dbl, dbl, ctypes.c_int, vp, sz, vp],
        "rpyw_tridiag_sqrt_coeffs": [ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32, dbl, ctypes.POINTER(dbl)],
        "rpy_wall_profile_enable": [ctypes.c_int],
        "rpy_wall_calibrate": [ctypes.c_int, i64, i32, vp, vp],
        "rpy_wall_set_shape": [ctypes.c_int, i64, i32, i32, i32, i32, i32, i32, i32],
        "rpy_wall_get_shape": [ctypes.c_int, i64, i32, ctypes.POINTER(i32)],
        "rpy_wall_profile_read": [ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.rpy_wall_noalloc_scratch_bytes.argtypes = []
    L.rpy_wall_noalloc_scratch_bytes.restype = sz
    L.rpy_wall_ts_state_bytes.argtypes = [i64, i32]
    L.rpy_wall_ts_state_bytes.restype = sz
    L.rpy_wall_workspace_bytes.argtypes = [ctypes.c_int, i64, i32, i32, i32, ctypes.c_int]
    L.rpy_wall_workspace_bytes.restype = sz
    L.rpyw_strerror.argtypes = [ctypes.c_int]
    L.rpyw_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, where: str, allow=(OK,)):
    if status not in allow:
        raise RpywError(status, where)
    return status


def _dev(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(device) -> int:
    """PyTorch's current HIP stream of the device (the raw handle; the
    public accessor builds a Stream object on every call, about 2 us)."""
    if _raw_stream is not None:
        return _raw_stream(device.index if device.index is not None else torch.cuda.current_device())
    return torch.cuda.current_stream(device).cuda_stream


_ws_bytes: dict = {}


def workspace_bytes(op: int, N: int, k: int = 1, max_iter: int = 0, n_bodies: int = 0,
                    precision: int = FP64) -> int:
    key = (op, N, k, max_iter, n_bodies, precision)
    b = _ws_bytes.get(key)
    if b is None:
        b = _ws_bytes[key] = int(lib().rpy_wall_workspace_bytes(op, N, k, max_iter, n_bodies, precision))
    return b


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


_scratch_ws: dict = {}


def _scratch(nbytes: int, device, stream: int) -> torch.Tensor:
    """A workspace kept per (device, stream) and grown on demand, for the
    single-call entry points whose workspace holds nothing between calls:
    calls on one stream run one after the other on the GPU, so they can share
    it (a replaced buffer goes back to PyTorch's stream-ordered allocator)."""
    key = (device.index, stream)
    t = _scratch_ws.get(key)
    if t is None or t.numel() < nbytes:
        t = _scratch_ws[key] = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    return t


def matvec(pos: torch.Tensor, force: torch.Tensor, a: float = 1.0, eta: float = 1.0,
           precision: int = FP64, out: torch.Tensor | None = None, box=None) -> torch.Tensor:
    """u = M(r) f for pos, force of shape (N, 3).  box = (Lx, Ly): the
    pseudo-periodic domain (minimum image plus 8 periodic images)."""
    N = pos.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(force, "force", (N, 3))
    out = torch.empty_like(force) if out is None else _dev(out, "out", (N, 3))
    if box is not None:
        return matvec_periodic(pos, force.view(1, N, 3), box, a, eta, precision, out.view(1, N, 3)).view(N, 3)
    st = _stream(pos.device)
    ws = _scratch(workspace_bytes(OP_MATVEC, N, 1, precision=precision), pos.device, st)
    _check(_lib.rpy_wall_matvec(pos.data_ptr(), force.data_ptr(), out.data_ptr(), N, a, eta, precision,
                                ws.data_ptr(), ws.numel(), st), "rpy_wall_matvec")
    return out


def matvec_noalloc(pos: torch.Tensor, force: torch.Tensor, a: float = 1.0, eta: float = 1.0,
                   precision: int = FP64, out: torch.Tensor | None = None) -> torch.Tensor:
    """u = M(r) f through the entry point that allocates nothing (its
    workspace is a fixed device array in the library; small N only)."""
    N = pos.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(force, "force", (N, 3))
    out = torch.empty_like(force) if out is None else _dev(out, "out", (N, 3))
    _check(lib().rpy_wall_matvec_noalloc(pos.data_ptr(), force.data_ptr(), out.data_ptr(), N, a, eta, precision,
                                         _stream(pos.device)), "rpy_wall_matvec_noalloc")
    return out


def matvec_multi(pos: torch.Tensor, F: torch.Tensor, a: float = 1.0, eta: float = 1.0,
                 precision: int = FP64, out: torch.Tensor | None = None) -> torch.Tensor:
    """U_l = M(r) F_l for F of shape (k, N, 3)."""
    N = pos.shape[0]
    k = F.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(F, "F", (k, N, 3))
    out = torch.empty_like(F) if out is None else _dev(out, "out", (k, N, 3))
    ws = _workspace(workspace_bytes(OP_MATVEC, N, k, precision=precision), pos.device)
    _check(lib().rpy_wall_matvec_multi(pos.data_ptr(), F.data_ptr(), out.data_ptr(), N, k, a, eta, precision,
                                       ws.data_ptr(), ws.numel(), _stream(pos.device)), "rpy_wall_matvec_multi")
    return out


def _offsets(offs) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(offs.cpu() if isinstance(offs, torch.Tensor) else offs,
                                          dtype=np.int64))
    return arr


def matvec_periodic(pos: torch.Tensor, F: torch.Tensor, box, a: float = 1.0, eta: float = 1.0,
                    precision: int = FP64, out: torch.Tensor | None = None) -> torch.Tensor:
    """U[l] = M F[l] in the pseudo-periodic cell box = (Lx, Ly); F, out: (k, N, 3)."""
    N = pos.shape[0]
    k = F.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(F, "F", (k, N, 3))
    out = torch.empty_like(F) if out is None else _dev(out, "out", (k, N, 3))
    ws = _workspace(workspace_bytes(OP_MATVEC, N, 1, precision=precision), pos.device)
    _check(lib().rpy_wall_matvec_periodic(pos.data_ptr(), F.data_ptr(), out.data_ptr(), N, k, a, eta,
                                          float(box[0]), float(box[1]), precision, ws.data_ptr(), ws.numel(),
                                          _stream(pos.device)), "rpy_wall_matvec_periodic")
    return out


def matvec_batched(pos: torch.Tensor, sys_offsets, F: torch.Tensor, a: float = 1.0, eta: float = 1.0,
                   precision: int = FP32C, out: torch.Tensor | None = None) -> torch.Tensor:
    """Independent systems in one persistent launch; F, out: (k, Ntot, 3)."""
    offs = _offsets(sys_offsets)
    S = offs.shape[0] - 1
    Ntot = pos.shape[0]
    k = F.shape[0]
    _dev(pos, "pos", (Ntot, 3))
    _dev(F, "F", (k, Ntot, 3))
    out = torch.empty_like(F) if out is None else _dev(out, "out", (k, Ntot, 3))
    ws = _workspace(workspace_bytes(OP_BATCHED, Ntot, k, 0, S, precision), pos.device)
    _check(lib().rpy_wall_matvec_batched(pos.data_ptr(), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), S,
                                         F.data_ptr(), out.data_ptr(), k, a, eta, precision, ws.data_ptr(),
                                         ws.numel(), _stream(pos.device)), "rpy_wall_matvec_batched")
    return out


def lanczos_sqrt(pos: torch.Tensor, W: torch.Tensor, a: float = 1.0, eta: float = 1.0, body_offsets=None,
                 tol: float = 1e-6, max_iter: int = 200, precision: int = FP64, out: torch.Tensor | None = None,
                 strict: bool = False, box=None):
    """Brownian blob displacements S W with S S^T = M by preconditioned
    Lanczos.  Returns (out (N,3), iterations, last relative change,
    converged flag).  strict=True raises when max_iter is reached."""
    N = pos.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(W, "W", (N, 3))
    out = torch.empty_like(W) if out is None else _dev(out, "out", (N, 3))
    if body_offsets is None:
        offs_p, nb = None, 0
    else:
        offs = _offsets(body_offsets)
        nb = offs.shape[0] - 1
        offs_p = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    ws = _workspace(workspace_bytes(OP_LANCZOS, N, 1, max_iter, nb, precision), pos.device)
    it = ctypes.c_int32(0)
    err = ctypes.c_double(0.0)
    if box is None:
        st = lib().rpy_wall_lanczos_sqrt(pos.data_ptr(), W.data_ptr(), out.data_ptr(), N, a, eta, offs_p, nb, tol,
                                         max_iter, precision, ws.data_ptr(), ws.numel(), ctypes.byref(it),
                                         ctypes.byref(err), _stream(pos.device))
    else:
        st = lib().rpy_wall_lanczos_sqrt_periodic(pos.data_ptr(), W.data_ptr(), out.data_ptr(), N, a, eta,
                                                  float(box[0]), float(box[1]), offs_p, nb, tol, max_iter,
                                                  precision, ws.data_ptr(), ws.numel(), ctypes.byref(it),
                                                  ctypes.byref(err), _stream(pos.device))
    _check(st, "rpy_wall_lanczos_sqrt", allow=(OK,) if strict else (OK, NOT_CONVERGED))
    return out, int(it.value), float(err.value), st == OK


def rigid_solve(pos: torch.Tensor, q: torch.Tensor, body_offsets, slip: torch.Tensor | None = None,
                force_torque: torch.Tensor | None = None, a: float = 1.0, eta: float = 1.0, tol: float = 1e-6,
                max_iter: int = 200, precision: int = FP64, strict: bool = False, box=None):
    """Rigid-multiblob mobility problem M lambda - K U = -slip,
    -K^T lambda = -F by block-preconditioned GMRES.  pos (N,3), q (nb,3)
    reference points, body_offsets host int64 [nb+1], slip (N,3) or None,
    force_torque (nb,6) or None.  Returns (lambda (N,3), U (nb,6) =
    (u, omega), iterations, relative residual estimate, converged flag)."""
    N = pos.shape[0]
    offs = _offsets(body_offsets)
    nb = offs.shape[0] - 1
    _dev(pos, "pos", (N, 3))
    _dev(q, "q", (nb, 3))
    if slip is not None:
        _dev(slip, "slip", (N, 3))
    if force_torque is not None:
        _dev(force_torque, "force_torque", (nb, 6))
    lam = torch.empty_like(pos)
    U = torch.empty((nb, 6), dtype=torch.float64, device=pos.device)
    ws = _workspace(workspace_bytes(OP_RIGID, N, 1, max_iter, nb, precision), pos.device)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    offs_p = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    sp = slip.data_ptr() if slip is not None else None
    fp = force_torque.data_ptr() if force_torque is not None else None
    if box is None:
        st = lib().rpy_wall_rigid_solve(pos.data_ptr(), q.data_ptr(), offs_p, nb, sp, fp, lam.data_ptr(),
                                        U.data_ptr(), N, a, eta, tol, max_iter, precision, ws.data_ptr(), ws.numel(),
                                        ctypes.byref(it), ctypes.byref(res), _stream(pos.device))
    else:
        st = lib().rpy_wall_rigid_solve_periodic(pos.data_ptr(), q.data_ptr(), offs_p, nb, sp, fp, lam.data_ptr(),
                                                 U.data_ptr(), N, a, eta, float(box[0]), float(box[1]), tol,
                                                 max_iter, precision, ws.data_ptr(), ws.numel(), ctypes.byref(it),
                                                 ctypes.byref(res), _stream(pos.device))
    _check(st, "rpy_wall_rigid_solve", allow=(OK,) if strict else (OK, NOT_CONVERGED))
    return lam, U, int(it.value), float(res.value), st == OK


def body_blobs(q: torch.Tensor, theta: torch.Tensor, ref: torch.Tensor, body_offsets) -> torch.Tensor:
    """Blob positions q_p + R(theta_p) rho_i; q (nb,3), theta (nb,4) unit
    quaternions (s, p), ref (N,3) body-frame positions."""
    offs = _offsets(body_offsets)
    nb, N = offs.shape[0] - 1, ref.shape[0]
    _dev(q, "q", (nb, 3))
    _dev(theta, "theta", (nb, 4))
    _dev(ref, "ref", (N, 3))
    pos = torch.empty_like(ref)
    ws = _workspace(8 * (nb + 1) + 1024, ref.device)
    _check(lib().rpy_wall_body_blobs(q.data_ptr(), theta.data_ptr(), ref.data_ptr(),
                                     offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nb, pos.data_ptr(), N,
                                     ws.data_ptr(), ws.numel(), _stream(ref.device)), "rpy_wall_body_blobs")
    return pos


def body_move(q: torch.Tensor, theta: torch.Tensor, U: torch.Tensor, h: float):
    """(q + h u, Rotate(theta, h omega)) for U (nb, 6)."""
    nb = q.shape[0]
    _dev(q, "q", (nb, 3))
    _dev(theta, "theta", (nb, 4))
    _dev(U, "U", (nb, 6))
    qo, to = torch.empty_like(q), torch.empty_like(theta)
    _check(lib().rpy_wall_body_move(q.data_ptr(), theta.data_ptr(), U.data_ptr(), h, nb, qo.data_ptr(),
                                    to.data_ptr(), _stream(q.device)), "rpy_wall_body_move")
    return qo, to


class TSStep:
    """The Trapezoidal Slip step (Alg. 2) as predict / correct around the
    caller's force evaluation.  Geometry: ref (N,3) body-frame blob
    positions, body_offsets (host), Lp (nb,) length scales; box = (Lx, Ly)
    for the pseudo-periodic cell."""

    def __init__(self, ref: torch.Tensor, body_offsets, Lp: torch.Tensor, kT: float, dt: float, delta: float,
                 a: float = 1.0, eta: float = 1.0, tol: float = 1e-3, max_iter: int = 200,
                 precision: int = FP64, box=None):
        self.offs = _offsets(body_offsets)
        self.nb, self.N = self.offs.shape[0] - 1, ref.shape[0]
        _dev(ref, "ref", (self.N, 3))
        _dev(Lp, "Lp", (self.nb,))
        self.ref, self.Lp = ref, Lp
        self.kT, self.dt, self.delta, self.a, self.eta = kT, dt, delta, a, eta
        self.tol, self.max_iter, self.precision = tol, max_iter, precision
        self.box = (0.0, 0.0) if box is None else (float(box[0]), float(box[1]))
        dev = ref.device
        sb = int(lib().rpy_wall_ts_state_bytes(self.N, self.nb))
        self.state = torch.empty(sb // 8 + 32, dtype=torch.float64, device=dev)
        self.ws = _workspace(workspace_bytes(OP_TS, self.N, 1, max_iter, self.nb, precision), dev)
        self.iters = []

    def _po(self):
        return self.offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def predict(self, q, theta, force_torque, Ws, Wn):
        """Returns (q~, theta~, blob positions at Q~)."""
        for t, n, sh in ((q, "q", (self.nb, 3)), (theta, "theta", (self.nb, 4)),
                         (force_torque, "force_torque", (self.nb, 6)), (Ws, "Ws", (self.N, 3)),
                         (Wn, "Wn", (self.N, 3))):
            _dev(t, n, sh)
        qt, tt, pt = torch.empty_like(q), torch.empty_like(theta), torch.empty_like(self.ref)
        it = (ctypes.c_int32 * 3)()
        st = lib().rpy_wall_ts_predict(q.data_ptr(), theta.data_ptr(), self.ref.data_ptr(), self._po(), self.nb,
                                       self.N, self.Lp.data_ptr(), force_torque.data_ptr(), Ws.data_ptr(),
                                       Wn.data_ptr(), self.kT, self.dt, self.delta, self.a, self.eta, self.box[0],
                                       self.box[1], self.tol, self.max_iter, self.precision, qt.data_ptr(),
                                       tt.data_ptr(), pt.data_ptr(), self.state.data_ptr(), self.state.numel() * 8,
                                       self.ws.data_ptr(), self.ws.numel(), it, _stream(q.device))
        _check(st, "rpy_wall_ts_predict", allow=(OK, NOT_CONVERGED))
        self.iters = list(it)
        return qt, tt, pt

    def correct(self, q, theta, q_tilde, theta_tilde, force_torque_tilde):
        """Returns (q^{n+1}, theta^{n+1})."""
        _dev(force_torque_tilde, "force_torque_tilde", (self.nb, 6))
        q1, t1 = torch.empty_like(q), torch.empty_like(theta)
        it = ctypes.c_int32(0)
        st = lib().rpy_wall_ts_correct(q.data_ptr(), theta.data_ptr(), q_tilde.data_ptr(), theta_tilde.data_ptr(),
                                       self.ref.data_ptr(), self._po(), self.nb, self.N,
                                       force_torque_tilde.data_ptr(), self.state.data_ptr(), self.dt, self.a,
                                       self.eta, self.box[0], self.box[1], self.tol, self.max_iter, self.precision,
                                       q1.data_ptr(), t1.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                       ctypes.byref(it), _stream(q.device))
        _check(st, "rpy_wall_ts_correct", allow=(OK, NOT_CONVERGED))
        self.iters.append(int(it.value))
        return q1, t1

    def step(self, q, theta, force_fn, Ws, Wn):
        """force_fn(q, theta, blob positions) -> (nb, 6) forces and torques
        at Q^n, predict, force_fn at Q~, correct."""
        F0 = force_fn(q, theta, body_blobs(q, theta, self.ref, self.offs))
        qt, tt, pt = self.predict(q, theta, F0, Ws, Wn)
        return self.correct(q, theta, qt, tt, force_fn(qt, tt, pt))


def emt_step(q: torch.Tensor, theta: torch.Tensor, ref: torch.Tensor, body_offsets, Lp: torch.Tensor,
             force_torque: torch.Tensor, Wf: torch.Tensor, Wt: torch.Tensor, Wn: torch.Tensor, kT: float, dt: float,
             delta: float, a: float = 1.0, eta: float = 1.0, tol: float = 1e-3, max_iter: int = 200,
             precision: int = FP64, box=None, scheme: str = "emt"):
    """One Euler-Maruyama step: the traction-corrected scheme (Alg. 1,
    scheme="emt") or the RFD scheme (Alg. 3, scheme="emrfd").  Returns
    (q^{n+1}, theta^{n+1}, iteration counts of the solves)."""
    offs = _offsets(body_offsets)
    nb, N = offs.shape[0] - 1, ref.shape[0]
    for t, n, sh in ((q, "q", (nb, 3)), (theta, "theta", (nb, 4)), (ref, "ref", (N, 3)), (Lp, "Lp", (nb,)),
                     (force_torque, "force_torque", (nb, 6)), (Wf, "Wf", (nb, 3)), (Wt, "Wt", (nb, 3)),
                     (Wn, "Wn", (N, 3))):
        _dev(t, n, sh)
    box = (0.0, 0.0) if box is None else (float(box[0]), float(box[1]))
    q1, t1 = torch.empty_like(q), torch.empty_like(theta)
    ws = _workspace(workspace_bytes(OP_TS, N, 1, max_iter, nb, precision), q.device)
    if scheme not in ("emt", "emrfd"):
        raise ValueError("scheme must be 'emt' or 'emrfd'")
    it = (ctypes.c_int32 * 4)()
    fn = lib().rpy_wall_emt_step if scheme == "emt" else lib().rpy_wall_emrfd_step
    st = fn(q.data_ptr(), theta.data_ptr(), ref.data_ptr(), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nb,
            N, Lp.data_ptr(), force_torque.data_ptr(), Wf.data_ptr(), Wt.data_ptr(), Wn.data_ptr(), kT, dt, delta, a,
            eta, box[0], box[1], tol, max_iter, precision, q1.data_ptr(), t1.data_ptr(), ws.data_ptr(), ws.numel(),
            it, _stream(q.device))
    _check(st, f"rpy_wall_{scheme}_step", allow=(OK, NOT_CONVERGED))
    return q1, t1, list(it)[:3 if scheme == "emt" else 4]


def matvec_vjp(pos: torch.Tensor, force: torch.Tensor, grad_vel: torch.Tensor, a: float = 1.0, eta: float = 1.0,
               precision: int = FP64, need_pos: bool = True, need_force: bool = True):
    """(grad_pos, grad_force) of L = sum grad_vel . M(pos) force."""
    N = pos.shape[0]
    for t, n in ((pos, "pos"), (force, "force"), (grad_vel, "grad_vel")):
        _dev(t, n, (N, 3))
    gp = torch.empty_like(pos) if need_pos else None
    gf = torch.empty_like(force) if need_force else None
    ws = _workspace(workspace_bytes(OP_VJP, N, 1, precision=precision), pos.device)
    _check(lib().rpy_wall_matvec_vjp(pos.data_ptr(), force.data_ptr(), grad_vel.data_ptr(),
                                     gp.data_ptr() if gp is not None else None,
                                     gf.data_ptr() if gf is not None else None, N, a, eta, precision,
                                     ws.data_ptr(), ws.numel(), _stream(pos.device)), "rpy_wall_matvec_vjp")
    return gp, gf


def divergence(pos: torch.Tensor, a: float = 1.0, eta: float = 1.0, precision: int = FP64) -> torch.Tensor:
    """Exact divergence of M, shape (N, 3)."""
    N = pos.shape[0]
    _dev(pos, "pos", (N, 3))
    out = torch.empty_like(pos)
    ws = _workspace(workspace_bytes(OP_DIVERGENCE, N, 1, precision=precision), pos.device)
    _check(lib().rpy_wall_divergence(pos.data_ptr(), out.data_ptr(), N, a, eta, precision, ws.data_ptr(),
                                     ws.numel(), _stream(pos.device)), "rpy_wall_divergence")
    return out


def autotune(pos: torch.Tensor, F: torch.Tensor, a: float = 1.0, eta: float = 1.0, precision: int = FP32C):
    """Time the launch-shape candidates on these inputs (F: (k, N, 3)) and
    keep the fastest for this precision and size class."""
    N = pos.shape[0]
    k = F.shape[0]
    _dev(pos, "pos", (N, 3))
    _dev(F, "F", (k, N, 3))
    U = torch.empty_like(F)
    ws = _workspace(workspace_bytes(OP_MATVEC, N, k, precision=precision), pos.device)
    _check(lib().rpy_wall_autotune(pos.data_ptr(), F.data_ptr(), U.data_ptr(), N, k, a, eta, precision,
                                   ws.data_ptr(), ws.numel(), _stream(pos.device)), "rpy_wall_autotune")


def set_shape(precision: int, N: int, k: int = 1, tpl: int = 1, tile: int = 256, kblk: int = 1, sym: int = 0,
              ipw: int = 4, mat: int = 0):
    """Fix the launch shape for products of this precision and size class
    (tpl=0 removes the override)."""
    _check(lib().rpy_wall_set_shape(precision, N, k, tpl, tile, kblk, sym, ipw, mat), "rpy_wall_set_shape")


def reset_shape(precision: int, N: int, k: int = 1):
    """Back to the built-in or tuned launch shape for this size class."""
    _check(lib().rpy_wall_set_shape(precision, N, k, 0, 0, 0, 0, 0, 0), "rpy_wall_set_shape")


def get_shape(precision: int, N: int, k: int = 1) -> dict:
    """Launch shape that products of this precision and size class use."""
    out = (ctypes.c_int32 * 6)()
    _check(lib().rpy_wall_get_shape(precision, N, k, out), "rpy_wall_get_shape")
    return dict(zip(("tpl", "tile", "kblk", "sym", "ipw", "mat"), list(out)))


def tridiag_sqrt_coeffs(alpha, beta, beta0: float) -> np.ndarray:
    """Host: c = beta0 Q Lambda^{1/2} Q^T e1 for tridiag(beta, alpha, beta)."""
    a_ = np.ascontiguousarray(alpha, dtype=np.float64)
    b_ = np.ascontiguousarray(beta, dtype=np.float64)
    k = a_.shape[0]
    c = np.empty(k)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().rpyw_tridiag_sqrt_coeffs(a_.ctypes.data_as(dp), b_.ctypes.data_as(dp) if k > 1 else None, k,
                                          float(beta0), c.ctypes.data_as(dp)), "rpyw_tridiag_sqrt_coeffs")
    return c


def calibrate(kind: int, blocks: int, iters: int, device=None) -> torch.Tensor:
    """Run the counter-calibration kernel (kind 0: FP32 FMAs, 1: FP64 FMAs;
    8 x iters FMA instructions per wave, 4 waves per block)."""
    dev = torch.device("cuda") if device is None else device
    out = torch.empty(blocks * 256, dtype=torch.float32 if kind == 0 else torch.float64, device=dev)
    _check(lib().rpy_wall_calibrate(kind, blocks, iters, out.data_ptr(), _stream(dev)), "rpy_wall_calibrate")
    return out


def profile_enable(flag: bool = True):
    lib().rpy_wall_profile_enable(1 if flag else 0)


def profile_read(reset: bool = True):
    """(summed pair-kernel milliseconds, launches, pair interactions)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    pairs = ctypes.c_double(0.0)
    _check(lib().rpy_wall_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pairs), 1 if reset else 0),
           "rpy_wall_profile_read")
    return ms.value, n.value, pairs.value


class RPYWallMatvec(torch.autograd.Function):
    """u = M(pos) force with a hand-written backward (the library's VJP)."""

    @staticmethod
    def forward(ctx, pos, force, a=1.0, eta=1.0, precision=FP64):
        ctx.save_for_backward(pos, force)
        ctx.params = (a, eta, precision)
        return matvec(pos.detach().contiguous(), force.detach().contiguous(), a, eta, precision)

    @staticmethod
    def backward(ctx, grad_vel):
        pos, force = ctx.saved_tensors
        a, eta, precision = ctx.params
        gp, gf = matvec_vjp(pos.detach().contiguous(), force.detach().contiguous(), grad_vel.contiguous(), a, eta,
                            precision, need_pos=ctx.needs_input_grad[0], need_force=ctx.needs_input_grad[1])
        return gp, gf, None, None, None


def rpy_wall_matvec(pos, force, a: float = 1.0, eta: float = 1.0, precision: int = FP64):
    """Differentiable u = M(pos) force."""
    return RPYWallMatvec.apply(pos, force, a, eta, precision)
