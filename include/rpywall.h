/*
 * rpywall.h - C ABI of librpywall.so: the wall-corrected Rotne-Prager-Yamakawa
 * blob mobility M(r) of arXiv:1709.02410 on MI355X (gfx950).
 *
 * Physics (Sec. II.A): blob i moves with velocity u_i = sum_j M_ij f_j under
 * forces f_j on all blobs j (self pair included); M_ij is the 3x3
 * Rotne-Prager-Yamakawa tensor for blobs of hydrodynamic radius a in a fluid
 * of viscosity eta, corrected for a no-slip wall at z = 0 (the
 * Rotne-Prager-Blake tensor; fluid in z > 0), with the overlap form for
 * blobs closer than 2a and a regularisation for blobs closer than a to the
 * wall that keeps M symmetric positive definite (Sec. IV, opening):
 *     z~ = max(z, a),  B = min(z/a, 1),  M_ij = B_i B_j Mhat(r~_i, r~_j).
 * Blobs with z <= 0 are accepted and use the same formula (B <= 0; M is then
 * singular at z = 0); positions are not scanned, NaN in gives NaN out.
 * Units: M scales with mu0 = 1/(6 pi eta a); k_B T and time steps are the
 * caller's (the Brownian velocity sqrt(2 k_B T / dt) M^{1/2} W of Sec. II.B
 * is the caller's scaling of the square root below).
 *
 * Conventions for every entry point:
 *   - Arrays named pos/force/vel/... are DEVICE pointers to FP64 row-major
 *     [N][3] arrays (x, y, z per blob); multi-RHS arrays are [k][N][3].
 *     Arrays documented as "host" are host pointers.
 *   - The caller owns every buffer.  Scratch memory: pass a device workspace
 *     `ws` of at least rpy_wall_workspace_bytes(...) bytes, 256-byte aligned;
 *     with ws == NULL the library takes stream-ordered scratch itself
 *     (hipMallocAsync/hipFreeAsync on `stream`).
 *   - `stream` is a hipStream_t (NULL: the default stream).  Calls are
 *     asynchronous on it unless stated otherwise.  Outputs must not alias
 *     inputs.  Calls that share a workspace must be ordered by the caller.
 *   - Arguments are validated on the host before any GPU work; a rejected
 *     call returns RPYW_EINVAL and launches nothing.  HIP failures return
 *     RPYW_EHIP.  No function throws or aborts.
 *   - precision: RPYW_FP64 evaluates every pair in FP64.  RPYW_FP32C
 *     evaluates pair terms in FP32 (positions carried as FP32 hi+lo pairs)
 *     and accumulates each target's sum with compensated (TwoSum) FP32
 *     arithmetic; inputs and outputs stay FP64.
 */
#ifndef RPYWALL_H
#define RPYWALL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rpyw_status {
    RPYW_OK = 0,
    RPYW_NOT_CONVERGED = 1, /* warning: max_iter reached, best iterate written */
    RPYW_EINVAL = -1,       /* invalid argument, nothing launched */
    RPYW_EHIP = -2,         /* HIP runtime error */
    RPYW_ENOMEM = -3,       /* workspace too small or allocation failed */
    RPYW_ENOTSPD = -4       /* a preconditioner block is not positive definite */
};

enum rpyw_precision { RPYW_FP64 = 0, RPYW_FP32C = 1 };

enum rpyw_op {
    RPYW_OP_MATVEC = 0,     /* rpy_wall_matvec / rpy_wall_matvec_multi */
    RPYW_OP_BATCHED = 1,    /* rpy_wall_matvec_batched (N = total blobs, n_bodies = S) */
    RPYW_OP_LANCZOS = 2,    /* rpy_wall_lanczos_sqrt */
    RPYW_OP_VJP = 3,        /* rpy_wall_matvec_vjp */
    RPYW_OP_DIVERGENCE = 4, /* rpy_wall_divergence */
    RPYW_OP_RIGID = 5,      /* rpy_wall_rigid_solve (and _periodic) */
    RPYW_OP_TS = 6          /* rpy_wall_ts_predict / _correct, rpy_wall_emt_step, _emrfd_step */
};

/* u = M(r) f  (Sec. II.A: the dense product whose cost dominates every
 * time step, evaluated by direct summation over all blob pairs).
 * pos, force, vel: device [N][3] FP64.  N >= 1, a > 0, eta > 0 finite. */
int rpy_wall_matvec(const double* pos, const double* force, double* vel, int64_t N, double a, double eta,
                    int precision, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same product as
 * rpy_wall_matvec (same kernels, launch shapes and results), with its
 * scratch memory in a fixed device array of rpy_wall_noalloc_scratch_bytes()
 * bytes (32 MiB) that the library holds on every GPU it runs on until the
 * process ends.  No allocation of any kind happens in the call.  N is
 * limited to problems whose workspace (rpy_wall_workspace_bytes with
 * RPYW_OP_MATVEC, k = 1, which is exact) fits that array: every N up to
 * 4096 blobs fits in both precisions (and many larger sizes, depending on
 * the launch plan); a larger workspace returns RPYW_ENOMEM and launches
 * nothing.  Every call on
 * one GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (different streams, threads or processes' streams not ordered by the
 * caller) race and must be ordered by the caller; the array keeps the last
 * call's contents, none of which a later call reads.  Arguments as for
 * rpy_wall_matvec. */
int rpy_wall_matvec_noalloc(const double* pos, const double* force, double* vel, int64_t N, double a, double eta,
                            int precision, void* stream);

/* Size of the fixed scratch array of rpy_wall_matvec_noalloc (host call). */
size_t rpy_wall_noalloc_scratch_bytes(void);

/* U_l = M(r) F_l for k right-hand sides sharing one geometry (one time step
 * needs M f, random-finite-difference probes and Lanczos vectors, Sec. III).
 * F, U: device [k][N][3].  Each pair's 3x3 block is evaluated once per RHS
 * block and contracted with every RHS in the block: by default on the matrix
 * cores for FP32C blocks of 8 or 16 (FP32 matrix products summed per source
 * tile, then compensated) and FP64 blocks of 16 (FP64 matrix products), the
 * block written out on the vector units; otherwise on the vector units.
 * 1 <= k <= 4096. */
int rpy_wall_matvec_multi(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a,
                          double eta, int precision, void* ws, size_t ws_bytes, void* stream);

/* Pseudo-periodic domain along the wall (the paper's dense suspensions,
 * Sec. IV.B): u = M f where every source blob enters at its minimum image
 * relative to the target and at the 8 periodic images around that one,
 * for the unit cell Lx x Ly in x and y (the wall stays at z = 0); the self
 * pair includes the blob's own 8 images.  The minimum image is the shift
 * by the nearest integer multiple of the cell (ties to even).  Positions
 * may lie outside the cell: they are wrapped into it first.  Evaluated by
 * the symmetric kernel, one right-hand side at a time (9 image blocks per
 * unordered pair).  F, U: device [k][N][3]; Lx, Ly > 0 in the units of
 * pos; other arguments as for rpy_wall_matvec_multi. */
int rpy_wall_matvec_periodic(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a,
                             double eta, double Lx, double Ly, int precision, void* ws, size_t ws_bytes,
                             void* stream);

/* S independent suspensions in one persistent launch: system s owns blobs
 * [sys_offsets[s], sys_offsets[s+1]) and blobs of different systems do not
 * interact.  sys_offsets: HOST int64 [S+1], sys_offsets[0] = 0, strictly
 * increasing.  pos: device [Ntot][3]; F, U: device [k][Ntot][3].  Work items
 * (system, target tile) are taken largest-first from an atomic counter;
 * FP32C blocks of 8 or more and FP64 blocks of 9 or more right-hand sides
 * run on the matrix cores (tiles of 64 targets), others on the vector units
 * (tiles of 256). */
int rpy_wall_matvec_batched(const double* pos, const int64_t* sys_offsets, int32_t S, const double* F,
                            double* U, int32_t k, double a, double eta, int precision, void* ws,
                            size_t ws_bytes, void* stream);

/* Brownian blob displacements out = S W with S S^T = M (Sec. II.B), by the
 * preconditioned Lanczos iteration:  out = L (L^-1 M L^-T)^{1/2} W, where L
 * is block diagonal, made of the Cholesky factors of the per-body dense
 * blocks M^(pp) that ignore other bodies (Sec. II.B, block-diagonal
 * preconditioner).  body_offsets: HOST int64 [n_bodies+1] (0 .. N, strictly
 * increasing, at most 42 blobs per body) or NULL for one 3x3 block per blob.
 * The iteration stops when |y_k - y_{k-1}| <= tol |y_k| (k >= 2) or on an
 * exact invariant subspace; full reorthogonalisation, FP64 Krylov vectors and
 * the host tridiagonal square root of rpyw_tridiag_sqrt_coeffs;
 * `precision` selects the pair arithmetic of the products by M.  pos, W,
 * out: device [N][3].  iters_out, err_est_out: HOST
 * (may be NULL) receive the iteration count and the last relative change.
 * Waits once per iteration for that step's scalars, so the iteration count
 * and the status are known on return; the final combination into `out`
 * (and up to two speculatively queued steps) are still stream-ordered on
 * `stream` then.  Returns RPYW_NOT_CONVERGED (best iterate written) if
 * max_iter is reached, RPYW_ENOTSPD if a block has no Cholesky factor (e.g.
 * a blob at z <= 0). */
int rpy_wall_lanczos_sqrt(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                          const int64_t* body_offsets, int32_t n_bodies, double tol, int32_t max_iter,
                          int precision, void* ws, size_t ws_bytes, int32_t* iters_out, double* err_est_out,
                          void* stream);

/* rpy_wall_lanczos_sqrt with the pseudo-periodic mobility of
 * rpy_wall_matvec_periodic (cell Lx x Ly).  The preconditioner blocks are
 * those of each body alone: its periodic images are ignored like the other
 * bodies. */
int rpy_wall_lanczos_sqrt_periodic(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                                   double Lx, double Ly, const int64_t* body_offsets, int32_t n_bodies, double tol,
                                   int32_t max_iter, int precision, void* ws, size_t ws_bytes, int32_t* iters_out,
                                   double* err_est_out, void* stream);

/* Mobility problem of rigid multiblobs (Sec. II.A, saddle-point system):
 *     M lambda - K U = -slip,    -K^T lambda = -F,
 * for the blob forces lambda and the body velocities U_p = (u_p, omega_p),
 * where (K U)_i = u_p + omega_p x (r_i - q_p) for blob i of body p and
 * K^T lambda is the force and the torque about q_p.  Solved by GMRES (no
 * restart, FP64 Arnoldi with two classical Gram-Schmidt passes, x0 = 0),
 * right-preconditioned with the block-diagonal operator of Sec. II.B
 * (interactions between distinct bodies dropped, each body's own dense
 * block M^(pp) kept, wall included), which is inverted exactly body by
 * body.  Stops when the residual estimate |b - A x| <= tol |b|,
 * b = [-slip; -F], or on breakdown.  Random slip slip = M^{1/2} W (from
 * rpy_wall_lanczos_sqrt) with F = 0 gives the Brownian body velocities
 * U = N^{1/2} W, N = (K^T M^-1 K)^-1 (Sec. II.B); kT and dt scalings are
 * the caller's.
 * pos: device [N][3]; q: device [n_bodies][3] reference points;
 * body_offsets: HOST int64 [n_bodies+1] (0 .. N, strictly increasing, at
 * most 42 blobs per body); slip: device [N][3] or NULL (zero);
 * force_torque: device [n_bodies][6] (F, T) or NULL (zero); outputs
 * lambda: device [N][3], U: device [n_bodies][6] (u, omega).  `precision`
 * selects the pair arithmetic of the products by M.  iters_out, res_out:
 * HOST (may be NULL) receive the iterations and the relative residual
 * estimate.  Waits once per iteration for that step's Hessenberg column;
 * the outputs are written stream-ordered after the call returns, as for
 * rpy_wall_lanczos_sqrt.  Returns RPYW_NOT_CONVERGED (iterate written) if
 * max_iter is reached,
 * RPYW_ENOTSPD if a body block has no Cholesky factor or a body's blobs do
 * not fix all six rigid motions (a single blob, a straight rod). */
int rpy_wall_rigid_solve(const double* pos, const double* q, const int64_t* body_offsets, int32_t n_bodies,
                         const double* slip, const double* force_torque, double* lambda, double* U, int64_t N,
                         double a, double eta, double tol, int32_t max_iter, int precision, void* ws,
                         size_t ws_bytes, int32_t* iters_out, double* res_out, void* stream);

/* rpy_wall_rigid_solve with the pseudo-periodic mobility of
 * rpy_wall_matvec_periodic (cell Lx x Ly); the preconditioner as for
 * rpy_wall_lanczos_sqrt_periodic. */
int rpy_wall_rigid_solve_periodic(const double* pos, const double* q, const int64_t* body_offsets, int32_t n_bodies,
                                  const double* slip, const double* force_torque, double* lambda, double* U,
                                  int64_t N, double a, double eta, double Lx, double Ly, double tol,
                                  int32_t max_iter, int precision, void* ws, size_t ws_bytes, int32_t* iters_out,
                                  double* res_out, void* stream);

/* Rigid-body kinematics (Sec. II: tracking point q_p and orientation
 * theta_p of every body; quaternion appendix: unit quaternions theta =
 * (s, p), rotated by quaternion multiplication).
 *
 * rpy_wall_body_blobs: blob positions r_i = q_p + R(theta_p) rho_i for blob i
 * of body p, with rho_i its position in the body frame.  q: device
 * [n_bodies][3]; theta: device [n_bodies][4] unit quaternions (s, px, py,
 * pz); ref: device [N][3] body-frame positions rho; body_offsets: HOST int64
 * [n_bodies+1] (0 .. N, strictly increasing); pos: device [N][3].
 * Asynchronous (the offsets go up through a library-owned pinned buffer,
 * so the caller's host array may be freed on return). */
int rpy_wall_body_blobs(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, double* pos, int64_t N, void* ws, size_t ws_bytes, void* stream);

/* rpy_wall_body_move: Q + h U for every body: q_out = q + h u, theta_out =
 * Rotate(theta, h omega), the quaternion of the rotation by the vector
 * h omega (angle |h omega|) times theta.  U: device [n_bodies][6] (u,
 * omega); other arrays as for rpy_wall_body_blobs.  Asynchronous. */
int rpy_wall_body_move(const double* q, const double* theta, const double* U, double h, int32_t n_bodies,
                       double* q_out, double* theta_out, void* stream);

/* One step of the Trapezoidal Slip scheme (Alg. 2), in two calls around the
 * caller's evaluation of forces and torques at the predicted configuration:
 *
 * rpy_wall_ts_predict, from Q^n = (q, theta), the forces and torques
 * force_torque = F(Q^n) (device [n_bodies][6], about q_p) and the Gaussian
 * vectors Ws (slip RFD) and Wn (Brownian), device [N][3]:
 *   W^D = [L_p W^s_p], W^F = [kT / L_p W^s_p] (Lp: device [n_bodies]);
 *   dQ^RFD: mobility problem with slip W^D and no force;
 *   Q+- = Q^n +- delta/2 dQ^RFD;  D^F = [K^T(Q+) - K^T(Q-)] W^F / delta,
 *   D^S = [M(Q+) - M(Q-)] W^F / delta (one batched product of both);
 *   sqrt(2 kT / dt) M^{1/2} W^n by the preconditioned Lanczos;
 *   U^n: mobility problem with that slip and force F^n;
 *   Q~ = Q^n + dt U^n -> q_tilde, theta_tilde and its blob positions
 *   pos_tilde (device [N][3]) for the caller's forces.
 * The quantities the corrector needs go to `state` (device, 256-byte
 * aligned, rpy_wall_ts_state_bytes(N, n_bodies) bytes, the caller's).
 * rpy_wall_ts_correct, with F(Q~) in force_torque_tilde: U~ from the
 * mobility problem at Q~ with slip 2 D^S + sqrt(2 kT / dt) M^{1/2} W^n and
 * force F(Q~) - 2 D^F, then Q^{n+1} = Q^n + dt/2 (U^n + U~) -> q_next,
 * theta_next (q, theta: Q^n again).
 *
 * Bodies: ref = body-frame blob positions, body_offsets HOST int64
 * [n_bodies+1], at most 42 blobs per body; the tracking points q_p are the
 * reference points of K.  Lx = Ly = 0: open domain; Lx, Ly > 0: the
 * pseudo-periodic cell of rpy_wall_matvec_periodic.  tol, max_iter: of every
 * iterative solve (Lanczos and GMRES); `precision`: pair arithmetic of the
 * products by M.  iters_out: HOST, may be NULL: predict writes 3 counts
 * (RFD solve, Lanczos, predictor solve), correct 1.  Both wait for the
 * iterative solves' per-iteration scalars; their device outputs are
 * stream-ordered (complete once `stream` reaches the end of the call's
 * work).  Returns RPYW_NOT_CONVERGED (step completed) if an iterative solve
 * hit max_iter, RPYW_ENOTSPD as the rigid solve does. */
size_t rpy_wall_ts_state_bytes(int64_t N, int32_t n_bodies);
int rpy_wall_ts_predict(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Ws,
                        const double* Wn, double kT, double dt, double delta, double a, double eta, double Lx,
                        double Ly, double tol, int32_t max_iter, int precision, double* q_tilde, double* theta_tilde,
                        double* pos_tilde, void* state, size_t state_bytes, void* ws, size_t ws_bytes,
                        int32_t* iters_out, void* stream);
int rpy_wall_ts_correct(const double* q, const double* theta, const double* q_tilde, const double* theta_tilde,
                        const double* ref, const int64_t* body_offsets, int32_t n_bodies, int64_t N,
                        const double* force_torque_tilde, const void* state, double dt, double a, double eta,
                        double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                        double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream);

/* One step of the Euler-Maruyama Traction scheme (Alg. 1):
 *   W^FT_p = kT [W^f_p / L_p, W^tau_p]  (Wf, Wt: device [n_bodies][3]);
 *   lambda^RFD, U^RFD: mobility problem with no slip and force W^FT;
 *   Q+- = Q^n +- delta/2 [L_p W^f_p, W^tau_p];
 *   D^F = [K^T(Q+) - K^T(Q-)] lambda^RFD / delta,
 *   D^S = [M(Q+) - M(Q-)] lambda^RFD / delta - [K(Q+) - K(Q-)] U^RFD / delta;
 *   U^n: mobility problem with slip D^S + sqrt(2 kT / dt) M^{1/2} W^n and
 *   force F^n - D^F (force_torque = F(Q^n));  Q^{n+1} = Q^n + dt U^n.
 * Other arguments as for rpy_wall_ts_predict; iters_out (HOST [3], may be
 * NULL): RFD solve, Lanczos, mobility solve.  Waits as
 * rpy_wall_ts_predict does; outputs stream-ordered. */
int rpy_wall_emt_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                      int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Wf,
                      const double* Wt, const double* Wn, double kT, double dt, double delta, double a, double eta,
                      double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                      double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream);

/* One step of the Euler-Maruyama RFD scheme (Alg. 3): U+- from the
 * mobility problems at Q+- = Q^n +- delta/2 [L_p W^f_p, W^tau_p] with no
 * slip and force W^FT (as for rpy_wall_emt_step); U^n from the mobility
 * problem at Q^n with slip sqrt(2 kT / dt) M^{1/2} W^n and force F^n;
 * Q^{n+1} = Q^n + dt (U^n + (U+ - U-) / delta).  Arguments as for
 * rpy_wall_emt_step; iters_out (HOST [4], may be NULL): the two RFD solves,
 * Lanczos, the mobility solve.  Waits as rpy_wall_ts_predict does; outputs
 * stream-ordered. */
int rpy_wall_emrfd_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Wf,
                        const double* Wt, const double* Wn, double kT, double dt, double delta, double a, double eta,
                        double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                        double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream);

/* Vector-Jacobian product of u = M(r) f for L = sum_i g_i . u_i
 * (derivatives of M drive the thermal drift, Sec. III):
 *   grad_force = M g  (M is symmetric),
 *   grad_pos_k = sum_j [g_k^T d1M(r_k, r_j) f_j + f_k^T d1M(r_k, r_j) g_j],
 * d1 = derivative in the first (target) argument; by reciprocity this is the
 * full gradient, self pair included.  Through the regularisation:
 * d z~/dz = 1{z >= a}, dB/dz = 1{z < a}/a; at the kinks (z = a, |r_ij| = 2a)
 * the upper branch is used, and coincident distinct blobs contribute zero.
 * pos, force, grad_vel: device [N][3]; grad_pos, grad_force: device [N][3]
 * or NULL (not computed; at least one must be non-NULL). */
int rpy_wall_matvec_vjp(const double* pos, const double* force, const double* grad_vel, double* grad_pos,
                        double* grad_force, int64_t N, double a, double eta, int precision, void* ws,
                        size_t ws_bytes, void* stream);

/* Exact divergence of M, div_i = sum_j sum_b dM_{ij,ab}/dr_{j,b}: the term
 * k_B T (d/dQ . M) that random finite differences estimate (Sec. III; the
 * self block contributes its total derivative).  pos, div: device [N][3]. */
int rpy_wall_divergence(const double* pos, double* div, int64_t N, double a, double eta, int precision,
                        void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace an entry point needs.  op: enum rpyw_op.  N: blobs
 * (total blobs for BATCHED), k: right-hand sides, max_iter: Lanczos or GMRES
 * bound, n_bodies: bodies for LANCZOS (0 = one per blob) and RIGID, or
 * systems S for BATCHED.
 * Returns 0 for invalid arguments. */
size_t rpy_wall_workspace_bytes(int op, int64_t N, int32_t k, int32_t max_iter, int32_t n_bodies,
                                int precision);

/* Static description of a status code (never NULL). */
const char* rpyw_strerror(int status);

/* Choose the launch shape (targets per lane, source tile, RHS block width,
 * symmetric or plain kernel) of the pair kernels for problems of this size
 * by timing the candidates on the given inputs; the result is kept for the
 * rest of the process and is used by every later call of the same precision
 * and size class.  Candidates are tried in a fixed order of preference and
 * a later one must be at least 1.5% faster to replace an earlier one, so
 * near-ties are resolved the same way from run to run.  Inputs as for
 * rpy_wall_matvec_multi (k RHS); blocks until the timing is done. */
int rpy_wall_autotune(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a,
                      double eta, int precision, void* ws, size_t ws_bytes, void* stream);

/* Fix the launch shape used for products of this precision and size class
 * (the class of N: floor(log2 N); of k: next power of two up to 16) instead
 * of the tuner's choice.  tpl: targets per lane (1, 2); tile: LDS tile (64,
 * 256); kblk: RHS block width (1..16; FP64 above 8 only with mat); sym: 1 or 2 selects
 * the symmetric kernel, which evaluates each unordered pair once and applies
 * it in both directions (kblk <= 4), over groups of 256 blobs (1) or of 64
 * blobs (2, more workgroups for small problems; taken for N <= 32768, else
 * groups of 256); ipw: source groups per workgroup of the symmetric kernel;
 * mat: 1 contracts the 3 x 3 pair blocks with the RHS block on the matrix
 * cores (kblk 8 or 16, in FP64 the only way to a block of 16; tpl, tile,
 * sym and ipw then do not apply), 0 on the vector units.  The batched
 * products do not read these shapes: they contract FP32C blocks of 8 or
 * more and FP64 blocks of 16 on the matrix cores.
 * Pseudo-periodic products always use the symmetric kernel, over groups of
 * 256 when sym is 1 and of 64 otherwise.  tpl = 0 removes the override (back to the tuner's or
 * the built-in choice).  Host-only, takes effect for later calls.
 * RPYW_EINVAL for values outside these sets. */
int rpy_wall_set_shape(int precision, int64_t N, int32_t k, int32_t tpl, int32_t tile, int32_t kblk, int32_t sym,
                       int32_t ipw, int32_t mat);

/* The launch shape later products of this precision and size class will
 * use: out6 = {tpl, tile, kblk, sym, ipw, mat} (HOST int32[6]), as for
 * rpy_wall_set_shape.  Host-only. */
int rpy_wall_get_shape(int precision, int64_t N, int32_t k, int32_t* out6);

/* Host-only: coefficients c = beta0 T^{1/2} e1 = beta0 Q Lambda^{1/2} Q^T e1
 * of the Lanczos iterate for the k x k symmetric tridiagonal T (diagonal
 * alpha[k], off-diagonal beta[k-1]) with eigendecomposition T = Q Lambda
 * Q^T, negative eigenvalues clamped to zero (Sec. II.B).  HOST arrays.  For
 * positive definite T of condition below 1e8 by an exponentially convergent
 * quadrature of T^{-1/2} (shifted tridiagonal solves; agrees with the
 * eigendecomposition to about 1e-15 of the largest coefficient); otherwise
 * the implicit symmetric QR algorithm with Wilkinson shifts.  Returns
 * RPYW_EINVAL for k < 1 or non-finite input, RPYW_NOT_CONVERGED if the QR
 * sweeps stall. */
int rpyw_tridiag_sqrt_coeffs(const double* alpha, const double* beta, int32_t k, double beta0,
                             double* c_out);

/* Instrumentation: when enabled, every launch of the pair kernels (the
 * O(N^2) products) is bracketed by HIP events on the launch stream and
 * rpy_wall_profile_read returns the summed kernel time (ms), the launch
 * count and the pair interactions evaluated (sum of k N^2) since the last
 * reset.  Reading synchronises the recorded events.  Not thread-safe. */
int rpy_wall_profile_enable(int enable);
int rpy_wall_profile_read(double* ms_total, int64_t* launches, double* pair_interactions, int reset);

/* Instrumentation: a kernel with an exactly known instruction count, for
 * calibrating hardware counters (rocprofv3 instruction and FLOP counts)
 * before they are used to report the FLOP rate of the pair kernels.
 * kind 0: FP32, 1: FP64.  `blocks` workgroups of 256 threads (4 waves) each
 * run `iters` x 8 fused multiply-add instructions per wave (8 independent
 * chains, operands in vector registers), then store one value per thread to
 * out (device, blocks x 256 floats or doubles, caller-owned).  Asynchronous
 * on stream.  1 <= blocks <= 2^20, iters >= 1. */
int rpy_wall_calibrate(int kind, int64_t blocks, int32_t iters, void* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RPYWALL_H */
