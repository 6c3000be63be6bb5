"""FP64 CPU oracle (Python side) for the wall-corrected RPY mobility.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; the pair formula lives in ``rpy_oracle.cpp``.

Contents (arXiv:1709.02410):
  * ``matvec``/``dense``/``pair_block``: the blob mobility M and u = M f
    (Sec. II.A), via the compiled C++ double loop.
  * ``vjp``/``divergence``: dual-number derivatives of M (Sec. III, the
    drift term that random finite differences estimate).
  * ``precond_blocks``: per-body dense blocks M^(pp) that ignore other
    bodies, and their Cholesky factors L_p (Sec. II.B, block-diagonal
    preconditioner).
  * ``lanczos_sqrt``: preconditioned Lanczos for M^{1/2} W (Sec. II.B),
    returning L (L^-1 M L^-T)^{1/2} W; ``dense_sqrt`` is the same root by
    a dense eigendecomposition for small N.
  * ``rfd_divergence``: the centred random-finite-difference estimate of
    the divergence of M (Sec. III, centred RFD with B = M and
    Delta P = Delta Q = W).
  * ``body_K``/``rigid_solve``/``body_mobility``: rigid multiblobs
    (Sec. II.A): the geometric matrix K, the saddle-point mobility problem
    solved densely, and N = (K^T M^-1 K)^-1.
  * ``rigid_gmres``: the same system by GMRES right-preconditioned with the
    per-body block-diagonal operator (Sec. II.B); used for iteration counts.
  * ``quat_rotate``/``body_blobs``/``body_move``/``ts_step``: body kinematics
    with unit quaternions (appendix on quaternions), one step of the
    Trapezoidal Slip scheme (Alg. 2), of the Euler-Maruyama Traction scheme
    (Alg. 1, ``emt_step``) and of the Euler-Maruyama RFD scheme (Alg. 3,
    ``emrfd_step``), with dense solves.
  * ``box=(Lx, Ly)`` on the products, dense matrices, roots and solves: the
    pseudo-periodic domain of the paper's suspensions (Sec. IV.B): each source
    at its minimum image plus the 8 periodic images around it.

Readings where the paper is silent (the Lanczos stopping rule, full
reorthogonalisation, breakdown handling) are stated in each docstring.
Parity unpinned: agreement with the authors' own blob-wall regularisation
and Lanczos stopping details (their sources are cited, not printed); the
properties the paper states for them are pinned by the tests.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpy_oracle.cpp")
_LIB = os.path.join(_HERE, "librpyoracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                        "-std=c++17", _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_pair_block.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
        lib.oracle_matvec.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      _lp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_dense.argtypes = [_dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_matvec_periodic.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, _lp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_dense_periodic.argtypes = [_dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_vjp.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   _dp, _dp, _lp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_divergence.argtypes = [_dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _dp,
                                          ctypes.c_int]
        for fn in ("oracle_pair_block", "oracle_matvec", "oracle_dense", "oracle_vjp", "oracle_divergence",
                   "oracle_matvec_periodic", "oracle_dense_periodic"):
            getattr(lib, fn).restype = None
        _lib = lib
    return _lib


def _c(x, dtype=np.float64):
    return np.ascontiguousarray(x, dtype=dtype)


def _p(x):
    return x.ctypes.data_as(_dp)


def mu0(a: float = 1.0, eta: float = 1.0) -> float:
    return 1.0 / (6.0 * math.pi * eta * a)


def pair_block(ri, rj, a: float = 1.0, eta: float = 1.0, part: int = 0) -> np.ndarray:
    """3x3 block M_ij (part 0, physical units) or its free (1) / wall (2)
    part in units of mu0, regularised heights, no B factors."""
    ri, rj = _c(ri), _c(rj)
    out = np.empty(9)
    _L().oracle_pair_block(_p(ri), _p(rj), a, eta, part, _p(out))
    return out.reshape(3, 3)


def matvec(pos, f, a: float = 1.0, eta: float = 1.0, rows=None, nthreads: int = 0, box=None) -> np.ndarray:
    """u = M f; with ``rows`` only those target rows (shape (len(rows), 3)).
    box = (Lx, Ly): pseudo-periodic domain (Sec. IV.B): every source at its
    minimum image and the 8 periodic images around it."""
    pos, f = _c(pos), _c(f)
    N = pos.shape[0]
    assert pos.shape == (N, 3) and f.shape == (N, 3)
    rp, nr = (None, 0) if rows is None else (_c(rows, np.int64), len(rows))
    out = np.empty((N if rows is None else nr, 3))
    rptr = None if rp is None else rp.ctypes.data_as(_lp)
    if box is None:
        _L().oracle_matvec(_p(pos), _p(f), _p(out), N, a, eta, rptr, nr, nthreads)
    else:
        _L().oracle_matvec_periodic(_p(pos), _p(f), _p(out), N, a, eta, float(box[0]), float(box[1]), rptr, nr,
                                    nthreads)
    return out


def dense(pos, a: float = 1.0, eta: float = 1.0, box=None) -> np.ndarray:
    """Dense 3N x 3N blob mobility matrix (small N); box as for matvec."""
    pos = _c(pos)
    N = pos.shape[0]
    out = np.empty((3 * N, 3 * N))
    if box is None:
        _L().oracle_dense(_p(pos), N, a, eta, _p(out))
    else:
        _L().oracle_dense_periodic(_p(pos), N, a, eta, float(box[0]), float(box[1]), _p(out))
    return out


def vjp(pos, f, g, a: float = 1.0, eta: float = 1.0, nthreads: int = 0, rows=None):
    """(grad_pos, grad_f) of L = sum_i g_i . (M(r) f)_i; with ``rows`` only
    those blobs' gradients (shape (len(rows), 3) each, in the order of rows)."""
    pos, f, g = _c(pos), _c(f), _c(g)
    N = pos.shape[0]
    rp, nr = (None, 0) if rows is None else (_c(rows, np.int64), len(rows))
    n = N if rows is None else nr
    gp = np.empty((n, 3))
    gf = np.empty((n, 3))
    rptr = None if rp is None else rp.ctypes.data_as(_lp)
    _L().oracle_vjp(_p(pos), _p(f), _p(g), N, a, eta, _p(gp), _p(gf), rptr, nr, nthreads)
    return gp, gf


def divergence(pos, a: float = 1.0, eta: float = 1.0, nthreads: int = 0) -> np.ndarray:
    """Exact divergence of M (sum over source blobs and force components)."""
    pos = _c(pos)
    N = pos.shape[0]
    out = np.empty((N, 3))
    _L().oracle_divergence(_p(pos), N, a, eta, _p(out), nthreads)
    return out


# ------------------------------------------------------------- square roots

def precond_blocks(pos, body_offsets=None, a: float = 1.0, eta: float = 1.0):
    """Block-diagonal preconditioner of Sec. II.B.

    For every body p: the dense block M^(pp) of its own blobs (other bodies
    ignored, wall included) and its lower Cholesky factor L_p.  With no body
    structure every blob is its own body (3x3 blocks).  Returns a list of
    (start, stop, L_p).  Raises numpy.linalg.LinAlgError if a block is not
    positive definite.
    """
    pos = _c(pos)
    N = pos.shape[0]
    offs = np.arange(N + 1) if body_offsets is None else np.asarray(body_offsets)
    out = []
    for p in range(len(offs) - 1):
        s, e = int(offs[p]), int(offs[p + 1])
        Mpp = dense(pos[s:e], a, eta)
        out.append((s, e, np.linalg.cholesky(Mpp)))
    return out


def _apply_blocks(blocks, v, mode: str) -> np.ndarray:
    """mode: 'L' -> L v, 'Linv' -> L^-1 v, 'LinvT' -> L^-T v (v flat 3N)."""
    out = np.empty_like(v)
    for s, e, Lp in blocks:
        seg = v[3 * s:3 * e]
        if mode == "L":
            out[3 * s:3 * e] = Lp @ seg
        elif mode == "Linv":
            out[3 * s:3 * e] = sla.solve_triangular(Lp, seg, lower=True)
        else:
            out[3 * s:3 * e] = sla.solve_triangular(Lp, seg, lower=True, trans="T")
    return out


def dense_sqrt(pos, W, body_offsets=None, a: float = 1.0, eta: float = 1.0, precondition: bool = True, box=None):
    """Dense reference root applied to W (flat 3N or (N,3)).

    precondition=True: L (L^-1 M L^-T)^{1/2} W with the block-Cholesky L,
    the root the preconditioned Lanczos converges to.  False: the symmetric
    M^{1/2} W.  Both satisfy S S^T = M (Sec. II.B).  With box, M is the
    pseudo-periodic mobility; the preconditioner blocks stay those of the
    bodies alone (their periodic images ignored like other bodies).
    """
    M = dense(pos, a, eta, box)
    w = np.asarray(W, dtype=np.float64).reshape(-1)
    if not precondition:
        lam, Q = np.linalg.eigh(M)
        return (Q @ (np.sqrt(np.clip(lam, 0.0, None)) * (Q.T @ w))).reshape(-1, 3)
    blocks = precond_blocks(pos, body_offsets, a, eta)
    n3 = M.shape[0]
    Linv = np.zeros((n3, n3))
    for s, e, Lp in blocks:
        Linv[3 * s:3 * e, 3 * s:3 * e] = sla.solve_triangular(Lp, np.eye(3 * (e - s)), lower=True)
    G = Linv @ M @ Linv.T
    G = 0.5 * (G + G.T)
    lam, Q = np.linalg.eigh(G)
    y = Q @ (np.sqrt(np.clip(lam, 0.0, None)) * (Q.T @ w))
    return _apply_blocks(blocks, y, "L").reshape(-1, 3)


def _tridiag_sqrt_coeffs(alpha, beta, beta0):
    """c = beta0 * Q Lambda^{1/2} Q^T e1 for T = tridiag(beta, alpha, beta),
    eigenvalues clamped at zero."""
    k = len(alpha)
    T = np.diag(alpha)
    if k > 1:
        T += np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    lam, Q = np.linalg.eigh(T)
    return beta0 * (Q @ (np.sqrt(np.clip(lam, 0.0, None)) * Q[0, :]))


def lanczos_sqrt(pos, W, body_offsets=None, a: float = 1.0, eta: float = 1.0, tol: float = 1e-6,
                 max_iter: int = 200, precondition: bool = True, matvec_fn=None, nthreads: int = 0, box=None):
    """Preconditioned Lanczos for the Brownian blob displacements (Sec. II.B).

    G = L^-1 M L^-T with the block-Cholesky factor L (identity when
    precondition=False).  beta0 = |W|, v1 = W / beta0; at step k:
    w = G v_k - beta_{k-1} v_{k-1}; alpha_k = v_k . w; w -= alpha_k v_k;
    full reorthogonalisation against all previous v, applied twice;
    y_k = beta0 V_k Q Lambda^{1/2} Q^T e1 from T_k = Q Lambda Q^T
    (negative eigenvalues clamped).  Stop when |y_k - y_{k-1}| <= tol |y_k|
    (k >= 2), or on breakdown beta_k <= 1e-14 (|alpha_k| + beta_{k-1}),
    which is an invariant subspace and counts as converged.  Otherwise
    beta_k = |w|, v_{k+1} = w / beta_k.  Returns (L y, iterations,
    last relative change, converged flag).
    """
    pos = _c(pos)
    w0 = np.asarray(W, dtype=np.float64).reshape(-1).copy()
    n3 = w0.shape[0]
    if precondition:
        blocks = precond_blocks(pos, body_offsets, a, eta)
    else:
        blocks = None

    def G(v):
        x = _apply_blocks(blocks, v, "LinvT") if blocks else v
        if matvec_fn is None:
            y = matvec(pos, x.reshape(-1, 3), a, eta, nthreads=nthreads, box=box).reshape(-1)
        else:
            y = np.asarray(matvec_fn(x.reshape(-1, 3))).reshape(-1)
        return _apply_blocks(blocks, y, "Linv") if blocks else y

    beta0 = float(np.linalg.norm(w0))
    if beta0 == 0.0:
        return np.zeros((n3 // 3, 3)), 0, 0.0, True
    V = np.zeros((n3, max_iter + 1))
    V[:, 0] = w0 / beta0
    alpha, beta = [], []
    y_prev = None
    rel = math.inf
    converged = False
    it = 0
    c = None
    for k in range(max_iter):
        it = k + 1
        w = G(V[:, k])
        if k > 0:
            w -= beta[k - 1] * V[:, k - 1]
        ak = float(V[:, k] @ w)
        w -= ak * V[:, k]
        for _ in range(2):
            w -= V[:, :k + 1] @ (V[:, :k + 1].T @ w)
        alpha.append(ak)
        bk = float(np.linalg.norm(w))
        c = _tridiag_sqrt_coeffs(np.array(alpha), np.array(beta), beta0)
        y = V[:, :k + 1] @ c
        if y_prev is not None:
            rel = float(np.linalg.norm(y - y_prev) / np.linalg.norm(y))
            if rel <= tol:
                converged = True
                break
        prev_b = beta[k - 1] if k > 0 else 0.0
        if bk <= 1e-14 * (abs(ak) + prev_b):
            converged = True
            break
        y_prev = y
        beta.append(bk)
        V[:, k + 1] = w / bk
    y = V[:, :len(c)] @ c
    out = _apply_blocks(blocks, y, "L") if blocks else y
    return out.reshape(-1, 3), it, rel, converged


def rfd_divergence(pos, delta: float, n_samples: int, seed: int, a: float = 1.0, eta: float = 1.0,
                   matvec_fn=None, nthreads: int = 0):
    """Centred random finite difference for the divergence of M (Sec. III):
    mean over samples of (1/delta) [M(r + delta W/2) - M(r - delta W/2)] W,
    W iid N(0,1) per blob component (kT = 1).  Returns (mean, std error)."""
    pos = _c(pos)
    rng = np.random.default_rng(seed)
    acc = np.zeros_like(pos)
    acc2 = np.zeros_like(pos)
    mv = matvec_fn or (lambda p, f: matvec(p, f, a, eta, nthreads=nthreads))
    for _ in range(n_samples):
        W = rng.standard_normal(pos.shape)
        s = (mv(pos + 0.5 * delta * W, W) - mv(pos - 0.5 * delta * W, W)) / delta
        acc += s
        acc2 += s * s
    mean = acc / n_samples
    var = np.maximum(acc2 / n_samples - mean * mean, 0.0)
    return mean, np.sqrt(var / n_samples)


# ------------------------------------------------------------- rigid bodies

def _body_ranges(N: int, body_offsets):
    offs = np.asarray(body_offsets, dtype=np.int64)
    if offs[0] != 0 or offs[-1] != N or np.any(np.diff(offs) < 1):
        raise ValueError("body_offsets must start at 0, end at N and be strictly increasing")
    return [(int(offs[p]), int(offs[p + 1])) for p in range(len(offs) - 1)]


def _cross_matrix(d) -> np.ndarray:
    """[d]_x with [d]_x v = d x v."""
    return np.array([[0.0, -d[2], d[1]], [d[2], 0.0, -d[0]], [-d[1], d[0], 0.0]])


def body_K(pos, q, body_offsets) -> np.ndarray:
    """Geometric matrix K of Sec. II.A (eq. K), dense (3N, 6 n_bodies).

    (K U)_i = u_p + omega_p x (r_i - q_p) for blob i of body p, with the
    body unknowns ordered (u_x, u_y, u_z, omega_x, omega_y, omega_z) and q_p
    the body's reference point.  omega x d = -[d]_x omega, so the blob's
    3x6 block is [I, -[r_i - q_p]_x].  K^T maps blob forces to the body
    force and torque about q_p.
    """
    pos = _c(pos)
    q = _c(q).reshape(-1, 3)
    ranges = _body_ranges(pos.shape[0], body_offsets)
    K = np.zeros((3 * pos.shape[0], 6 * len(ranges)))
    for p, (s, e) in enumerate(ranges):
        for i in range(s, e):
            K[3 * i:3 * i + 3, 6 * p:6 * p + 3] = np.eye(3)
            K[3 * i:3 * i + 3, 6 * p + 3:6 * p + 6] = -_cross_matrix(pos[i] - q[p])
    return K


def _rigid_rhs(N: int, nb: int, slip, FT) -> np.ndarray:
    s = np.zeros(3 * N) if slip is None else np.asarray(slip, dtype=np.float64).reshape(-1)
    F = np.zeros(6 * nb) if FT is None else np.asarray(FT, dtype=np.float64).reshape(-1)
    return np.concatenate([-s, -F])


def rigid_solve(pos, q, body_offsets, slip=None, FT=None, a: float = 1.0, eta: float = 1.0, box=None):
    """Mobility problem of rigid multiblobs (Sec. II.A, saddle-point system):

        [ M   -K ] [lambda]   [-slip]
        [-K^T  0 ] [  U   ] = [ -F  ]

    assembled densely (M from the pair formula, K from body_K) and solved by
    LU.  slip: (N, 3) prescribed slip (None = 0); FT: (n_bodies, 6) force
    and torque about q_p (None = 0).  Returns (lambda (N, 3), U (nb, 6)).
    """
    pos = _c(pos)
    N = pos.shape[0]
    K = body_K(pos, q, body_offsets)
    nb = K.shape[1] // 6
    M = dense(pos, a, eta, box)
    A = np.block([[M, -K], [-K.T, np.zeros((6 * nb, 6 * nb))]])
    x = np.linalg.solve(A, _rigid_rhs(N, nb, slip, FT))
    return x[:3 * N].reshape(N, 3), x[3 * N:].reshape(nb, 6)


def body_mobility(pos, q, body_offsets, a: float = 1.0, eta: float = 1.0, box=None) -> np.ndarray:
    """Body mobility N = (K^T M^-1 K)^-1 (Sec. II.A, eq. N_def), through a
    dense Cholesky factorisation of M.  (6 nb, 6 nb)."""
    K = body_K(pos, q, body_offsets)
    cf = sla.cho_factor(dense(pos, a, eta, box), lower=True)
    return np.linalg.inv(K.T @ sla.cho_solve(cf, K))


def rigid_gmres(pos, q, body_offsets, slip=None, FT=None, a: float = 1.0, eta: float = 1.0,
                tol: float = 1e-8, max_iter: int = 200, precondition: bool = True, matvec_fn=None,
                nthreads: int = 0, box=None):
    """The saddle-point system of rigid_solve by GMRES, right-preconditioned
    with the block-diagonal approximation of Sec. II.B (interactions between
    distinct bodies dropped, each body's own block M^(pp) kept, wall
    included), i.e. the per-body saddle-point operator

        P = [ diag_p M^(pp)   -K ]
            [ -K^T             0 ],

    applied exactly body by body (dense LU of each small system).

    Plain GMRES (Saad): x0 = 0, Arnoldi on A P^-1 from b / |b| with
    Gram-Schmidt applied twice per step, least-squares residual
    min |beta e1 - H y| after every step; stop when it is <= tol |b| or on
    breakdown.  x = P^-1 V y.  Returns (lambda (N, 3), U (nb, 6),
    iterations, relative residual estimate, converged).
    """
    pos = _c(pos)
    N = pos.shape[0]
    ranges = _body_ranges(N, body_offsets)
    nb = len(ranges)
    q = _c(q).reshape(-1, 3)
    K = body_K(pos, q, body_offsets)
    b = _rigid_rhs(N, nb, slip, FT)
    n = b.shape[0]
    small = []
    for p, (s, e) in enumerate(ranges):
        Kp = K[3 * s:3 * e, 6 * p:6 * p + 6]
        Mpp = dense(pos[s:e], a, eta)
        small.append(np.block([[Mpp, -Kp], [-Kp.T, np.zeros((6, 6))]]))

    def Pinv(v):
        if not precondition:
            return v.copy()
        out = np.empty_like(v)
        for p, (s, e) in enumerate(ranges):
            rhs = np.concatenate([v[3 * s:3 * e], v[3 * N + 6 * p:3 * N + 6 * p + 6]])
            sol = np.linalg.solve(small[p], rhs)
            out[3 * s:3 * e] = sol[:3 * (e - s)]
            out[3 * N + 6 * p:3 * N + 6 * p + 6] = sol[3 * (e - s):]
        return out

    def A(x):
        lam, U = x[:3 * N], x[3 * N:]
        if matvec_fn is None:
            Ml = matvec(pos, lam.reshape(-1, 3), a, eta, nthreads=nthreads, box=box).reshape(-1)
        else:
            Ml = np.asarray(matvec_fn(lam.reshape(-1, 3))).reshape(-1)
        return np.concatenate([Ml - K @ U, -(K.T @ lam)])

    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros((N, 3)), np.zeros((nb, 6)), 0, 0.0, True
    V = np.zeros((n, max_iter + 1))
    H = np.zeros((max_iter + 1, max_iter))
    V[:, 0] = b / beta
    res = 1.0
    converged = False
    k = 0
    y = np.zeros(0)
    for k in range(1, max_iter + 1):
        w = A(Pinv(V[:, k - 1]))
        for _ in range(2):
            h = V[:, :k].T @ w
            w -= V[:, :k] @ h
            H[:k, k - 1] += h
        H[k, k - 1] = np.linalg.norm(w)
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
        res = float(np.linalg.norm(e1 - H[:k + 1, :k] @ y)) / beta
        if res <= tol or H[k, k - 1] <= 1e-14 * beta:
            converged = True
            break
        V[:, k] = w / H[k, k - 1]
    x = Pinv(V[:, :len(y)] @ y)
    return x[:3 * N].reshape(N, 3), x[3 * N:].reshape(nb, 6), k, res, converged


# ------------------------------------------------------------- integrators

def quat_mul(a, b) -> np.ndarray:
    """Quaternion product of (s, p) quaternions, rows of (n, 4) arrays:
    (s1 s2 - p1.p2, s1 p2 + s2 p1 + p1 x p2)."""
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    s1, p1, s2, p2 = a[:, :1], a[:, 1:], b[:, :1], b[:, 1:]
    return np.concatenate([s1 * s2 - (p1 * p2).sum(1, keepdims=True), s1 * p2 + s2 * p1 + np.cross(p1, p2)], 1)


def quat_rotate(theta, phi) -> np.ndarray:
    """Rotate(theta, phi) of the quaternion appendix: the orientation theta
    (rows (s, p), unit norm) turned by the rotation vector phi (angle |phi|
    about phi / |phi|), i.e. theta' = [cos(|phi|/2), sin(|phi|/2) phi/|phi|] theta."""
    phi = np.atleast_2d(np.asarray(phi, dtype=np.float64))
    ang = np.linalg.norm(phi, axis=1, keepdims=True)
    axis = np.divide(phi, ang, out=np.zeros_like(phi), where=ang > 0)
    r = np.concatenate([np.cos(0.5 * ang), np.sin(0.5 * ang) * axis], 1)
    return quat_mul(r, theta)


def quat_matrix(theta) -> np.ndarray:
    """Rotation matrices (n, 3, 3) of unit quaternions (s, p):
    R = (s^2 - p.p) I + 2 p p^T + 2 s [p]_x."""
    theta = np.atleast_2d(theta)
    s, p = theta[:, 0], theta[:, 1:]
    R = (s * s - (p * p).sum(1))[:, None, None] * np.eye(3) + 2.0 * p[:, :, None] * p[:, None, :]
    return R + 2.0 * s[:, None, None] * np.stack([_cross_matrix(v) for v in p])


def body_blobs(q, theta, ref, body_offsets) -> np.ndarray:
    """Blob positions r_i = q_p + R(theta_p) rho_i of every body, with rho_i
    the blob's position in the body frame (ref, (N, 3))."""
    q = _c(q).reshape(-1, 3)
    ref = _c(ref)
    R = quat_matrix(theta)
    out = np.empty_like(ref)
    for p, (s, e) in enumerate(_body_ranges(ref.shape[0], body_offsets)):
        out[s:e] = q[p] + ref[s:e] @ R[p].T
    return out


def body_move(q, theta, U, scale: float):
    """Q + scale U for bodies: q + scale u, Rotate(theta, scale omega)."""
    U = np.asarray(U, dtype=np.float64).reshape(-1, 6)
    return _c(q).reshape(-1, 3) + scale * U[:, :3], quat_rotate(theta, scale * U[:, 3:])


def ts_step(q, theta, ref, body_offsets, Lp, force_fn, Ws, Wn, kT: float, dt: float, delta: float,
            a: float = 1.0, eta: float = 1.0, box=None):
    """One Trapezoidal Slip step (Alg. 2), with dense linear algebra.

    force_fn(q, theta) -> (n_bodies, 6) forces and torques; Ws, Wn: (N, 3)
    Gaussian vectors of the slip RFD and of the Brownian increment; Lp:
    body length scales.  Steps, in the algorithm's order:
      1a. W^D = [L_p W^s_p], W^F = [kT / L_p W^s_p];
      1b. RFD displacement problem with slip W^D, F = 0 -> dQ^RFD;
      1c. Q+- = Q^n +- delta/2 dQ^RFD;
      1d. D^F = [K^T(Q+) - K^T(Q-)] W^F / delta,
          D^S = [M(Q+) - M(Q-)] W^F / delta;
      2.  (M^{1/2})^n W^n: the block-preconditioned root L (L^-1 M L^-T)^{1/2} W^n;
      3.  predictor: slip sqrt(2 kT / dt) M^{1/2} W^n, force F^n -> U^n;
      4.  Q~ = Q^n + dt U^n;
      5.  corrector at Q~: slip 2 D^S + sqrt(2 kT / dt) M^{1/2} W^n,
          force F(Q~) - 2 D^F -> U~;
      6.  Q^{n+1} = Q^n + dt/2 (U^n + U~).
    Rigid solves are rigid_solve (dense LU) at the configuration named; body
    reference points are the tracking points q_p.  Returns (q1, theta1,
    intermediates dict).
    """
    ranges = _body_ranges(_c(ref).shape[0], body_offsets)
    Lb = np.concatenate([np.full(e - s, float(Lp[p])) for p, (s, e) in enumerate(ranges)])[:, None]
    WD = Lb * np.asarray(Ws)
    WF = kT / Lb * np.asarray(Ws)
    pos0 = body_blobs(q, theta, ref, body_offsets)
    _, dQ = rigid_solve(pos0, q, body_offsets, WD, None, a, eta, box)
    qp, tp = body_move(q, theta, dQ, 0.5 * delta)
    qm, tm = body_move(q, theta, dQ, -0.5 * delta)
    posp, posm = body_blobs(qp, tp, ref, body_offsets), body_blobs(qm, tm, ref, body_offsets)
    DF = (body_K(posp, qp, body_offsets).T @ WF.reshape(-1) - body_K(posm, qm, body_offsets).T @ WF.reshape(-1))
    DF = (DF / delta).reshape(-1, 6)
    DS = (matvec(posp, WF, a, eta, box=box) - matvec(posm, WF, a, eta, box=box)) / delta
    root = dense_sqrt(pos0, Wn, body_offsets, a, eta, box=box)
    c = math.sqrt(2.0 * kT / dt)
    F0 = force_fn(q, theta)
    _, U0 = rigid_solve(pos0, q, body_offsets, c * root, F0, a, eta, box)
    qt, tt = body_move(q, theta, U0, dt)
    post = body_blobs(qt, tt, ref, body_offsets)
    Ft = force_fn(qt, tt)
    _, Ut = rigid_solve(post, qt, body_offsets, 2.0 * DS + c * root, Ft - 2.0 * DF, a, eta, box)
    q1, t1 = body_move(q, theta, U0 + Ut, 0.5 * dt)
    return q1, t1, {"dQ_rfd": dQ, "DF": DF, "DS": DS, "root": root, "U0": U0, "q_tilde": qt, "theta_tilde": tt,
                    "U_tilde": Ut, "pos_plus": posp, "pos_minus": posm, "WF": WF}


def emt_step(q, theta, ref, body_offsets, Lp, FT, Wf, Wt, Wn, kT: float, dt: float, delta: float,
             a: float = 1.0, eta: float = 1.0, box=None):
    """One Euler-Maruyama Traction step (Alg. 1), with dense linear algebra.

    FT: (n_bodies, 6) forces and torques at Q^n; Wf, Wt: (n_bodies, 3)
    Gaussian vectors of the traction RFD; Wn: (N, 3) Brownian.  Steps:
      1a. W^FT_p = kT [W^f_p / L_p, W^tau_p];
      1b. RFD mobility problem with no slip and force W^FT -> lambda^RFD,
          U^RFD;
      1c. Q+- = Q^n +- delta/2 [L_p W^f_p, W^tau_p];
      1d. D^F = [K^T(Q+) - K^T(Q-)] lambda^RFD / delta,
          D^S = [M(Q+) - M(Q-)] lambda^RFD / delta
                - [K(Q+) - K(Q-)] U^RFD / delta;
      2.  (M^{1/2})^n W^n (block-preconditioned root);
      3.  slip D^S + sqrt(2 kT / dt) M^{1/2} W^n, force F^n - D^F -> U^n;
      4.  Q^{n+1} = Q^n + dt U^n.
    Returns (q1, theta1, intermediates dict)."""
    Lp = np.asarray(Lp, dtype=np.float64)
    WFT = kT * np.concatenate([np.asarray(Wf) / Lp[:, None], np.asarray(Wt)], 1)
    pos0 = body_blobs(q, theta, ref, body_offsets)
    lam_r, U_r = rigid_solve(pos0, q, body_offsets, None, WFT, a, eta, box)
    dQ = np.concatenate([Lp[:, None] * np.asarray(Wf), np.asarray(Wt)], 1)
    qp, tp = body_move(q, theta, dQ, 0.5 * delta)
    qm, tm = body_move(q, theta, dQ, -0.5 * delta)
    posp, posm = body_blobs(qp, tp, ref, body_offsets), body_blobs(qm, tm, ref, body_offsets)
    Kp, Km = body_K(posp, qp, body_offsets), body_K(posm, qm, body_offsets)
    lam_flat = lam_r.reshape(-1)
    DF = ((Kp.T @ lam_flat - Km.T @ lam_flat) / delta).reshape(-1, 6)
    DS = (matvec(posp, lam_r, a, eta, box=box) - matvec(posm, lam_r, a, eta, box=box)) / delta
    DS -= ((Kp @ U_r.reshape(-1) - Km @ U_r.reshape(-1)) / delta).reshape(-1, 3)
    root = dense_sqrt(pos0, Wn, body_offsets, a, eta, box=box)
    c = math.sqrt(2.0 * kT / dt)
    _, U0 = rigid_solve(pos0, q, body_offsets, DS + c * root, np.asarray(FT) - DF, a, eta, box)
    q1, t1 = body_move(q, theta, U0, dt)
    return q1, t1, {"lam_rfd": lam_r, "U_rfd": U_r, "dQ": dQ, "DF": DF, "DS": DS, "root": root, "U0": U0,
                    "pos_plus": posp, "pos_minus": posm}


def emrfd_step(q, theta, ref, body_offsets, Lp, FT, Wf, Wt, Wn, kT: float, dt: float, delta: float,
               a: float = 1.0, eta: float = 1.0, box=None):
    """One Euler-Maruyama RFD step (Alg. 3), with dense linear algebra:
      1. W^FT_p = kT [W^f_p / L_p, W^tau_p]; Q+- = Q^n +- delta/2 [L_p W^f_p, W^tau_p];
         U+- from the mobility problems at Q+- with no slip and force W^FT;
      2. (M^{1/2})^n W^n (block-preconditioned root);
      3. U^n: slip sqrt(2 kT / dt) M^{1/2} W^n, force F^n;
      4. Q^{n+1} = Q^n + dt (U^n + (U+ - U-) / delta).
    Returns (q1, theta1, intermediates dict)."""
    Lp = np.asarray(Lp, dtype=np.float64)
    WFT = kT * np.concatenate([np.asarray(Wf) / Lp[:, None], np.asarray(Wt)], 1)
    dQ = np.concatenate([Lp[:, None] * np.asarray(Wf), np.asarray(Wt)], 1)
    qp, tp = body_move(q, theta, dQ, 0.5 * delta)
    qm, tm = body_move(q, theta, dQ, -0.5 * delta)
    _, Up = rigid_solve(body_blobs(qp, tp, ref, body_offsets), qp, body_offsets, None, WFT, a, eta, box)
    _, Um = rigid_solve(body_blobs(qm, tm, ref, body_offsets), qm, body_offsets, None, WFT, a, eta, box)
    pos0 = body_blobs(q, theta, ref, body_offsets)
    root = dense_sqrt(pos0, Wn, body_offsets, a, eta, box=box)
    _, U0 = rigid_solve(pos0, q, body_offsets, math.sqrt(2.0 * kT / dt) * root, FT, a, eta, box)
    q1, t1 = body_move(q, theta, U0 + (Up - Um) / delta, dt)
    return q1, t1, {"U_plus": Up, "U_minus": Um, "U0": U0, "WFT": WFT, "q_plus": qp, "theta_plus": tp,
                    "q_minus": qm, "theta_minus": tm}
