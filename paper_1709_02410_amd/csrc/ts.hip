// Temporal integrators for rigid multiblobs (arXiv:1709.02410, Sec. III and Appendix A).
//
// Trapezoidal Slip (T-S, Alg. 2, with the slip-corrected random finite
// difference), split in two calls around the caller's force evaluation:
//
//   predict: W^D = [L_p W^s_p], W^F = [kT / L_p W^s_p];
//            dQ^RFD from the saddle-point problem with slip W^D, F = 0;
//            Q+- = Q^n +- delta/2 dQ^RFD;
//            D^F = [K^T(Q+) - K^T(Q-)] W^F / delta,
//            D^S = [M(Q+) - M(Q-)] W^F / delta (the two configurations as
//            two systems of one batched product);
//            c M^{1/2} W^n by the preconditioned Lanczos, c = sqrt(2 kT / dt);
//            U^n from the saddle-point problem with slip c M^{1/2} W^n and
//            force F^n; Q~ = Q^n + dt U^n.
//   correct: U~ at Q~ with slip 2 D^S + c M^{1/2} W^n and force F(Q~) - 2 D^F;
//            Q^{n+1} = Q^n + dt/2 (U^n + U~).
//
// Euler-Maruyama Traction (EM-T, Alg. 1, with the traction-corrected random
// finite difference), one call: W^FT_p = kT [W^f_p / L_p, W^tau_p]; the RFD
// problem with no slip and force W^FT gives lambda^RFD, U^RFD; Q+- = Q^n +-
// delta/2 [L_p W^f, W^tau]; D^F = [K^T(Q+) - K^T(Q-)] lambda^RFD / delta,
// D^S = [M(Q+) - M(Q-)] lambda^RFD / delta - [K(Q+) - K(Q-)] U^RFD / delta;
// U^n from slip D^S + c M^{1/2} W^n and force F^n - D^F; Q^{n+1} = Q^n + dt U^n.
//
// Euler-Maruyama RFD (EM-RFD, Alg. 3), one call: U+- from the mobility
// problems at Q+- = Q^n +- delta/2 [L_p W^f, W^tau] with no slip and force
// W^FT; U^n at Q^n from slip c M^{1/2} W^n and force F^n;
// Q^{n+1} = Q^n + dt (U^n + (U+ - U-) / delta).
//
// Bodies: tracking point q_p and unit quaternion theta_p = (s, p); blob i
// of body p sits at q_p + R(theta_p) rho_i with rho_i its body-frame
// position; Q + h U moves q_p by h u_p and rotates theta_p by the rotation
// vector h omega_p (quaternion appendix, Rotate).  The tracking points are
// the reference points of K.
#include <cmath>
#include <vector>

#include "rpyw_internal.h"

namespace rpyw {

namespace {

constexpr int kTT = 64;  // threads per body

// r_i = q_p + R(theta_p) rho_i,  R rho = (s^2 - p.p) rho + 2 (p.rho) p + 2 s p x rho.
__global__ __launch_bounds__(kTT) void body_blobs_kernel(const double* __restrict__ q,
                                                        const double* __restrict__ th,
                                                        const double* __restrict__ ref,
                                                        const int* __restrict__ bofs, double* __restrict__ pos) {
    const int b = blockIdx.x;
    const double s = th[4 * b], px = th[4 * b + 1], py = th[4 * b + 2], pz = th[4 * b + 3];
    const double c0 = s * s - (px * px + py * py + pz * pz);
    for (int i = bofs[b] + threadIdx.x; i < bofs[b + 1]; i += blockDim.x) {
        const double rx = ref[3 * i], ry = ref[3 * i + 1], rz = ref[3 * i + 2];
        const double pr = 2.0 * (px * rx + py * ry + pz * rz);
        pos[3 * i] = q[3 * b] + c0 * rx + pr * px + 2.0 * s * (py * rz - pz * ry);
        pos[3 * i + 1] = q[3 * b + 1] + c0 * ry + pr * py + 2.0 * s * (pz * rx - px * rz);
        pos[3 * i + 2] = q[3 * b + 2] + c0 * rz + pr * pz + 2.0 * s * (px * ry - py * rx);
    }
}

// q' = q + h u;  theta' = [cos(|phi|/2), sin(|phi|/2) phi/|phi|] theta, phi = h omega.
// U may be the sum of two velocity arrays (U2 non-null).
__global__ void body_move_kernel(const double* __restrict__ q, const double* __restrict__ th,
                                 const double* __restrict__ U, const double* __restrict__ U2, double h, int nb,
                                 double* __restrict__ qo, double* __restrict__ tho) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double u[6];
    for (int c = 0; c < 6; ++c) u[c] = U[6 * b + c] + (U2 ? U2[6 * b + c] : 0.0);
    for (int c = 0; c < 3; ++c) qo[3 * b + c] = q[3 * b + c] + h * u[c];
    const double fx = h * u[3], fy = h * u[4], fz = h * u[5];
    const double ang = sqrt(fx * fx + fy * fy + fz * fz);
    double rs = 1.0, rx = 0.0, ry = 0.0, rz = 0.0;
    if (ang > 0.0) {
        const double k = sin(0.5 * ang) / ang;
        rs = cos(0.5 * ang);
        rx = k * fx;
        ry = k * fy;
        rz = k * fz;
    }
    const double s = th[4 * b], px = th[4 * b + 1], py = th[4 * b + 2], pz = th[4 * b + 3];
    tho[4 * b] = rs * s - (rx * px + ry * py + rz * pz);
    tho[4 * b + 1] = rs * px + s * rx + (ry * pz - rz * py);
    tho[4 * b + 2] = rs * py + s * ry + (rz * px - rx * pz);
    tho[4 * b + 3] = rs * pz + s * rz + (rx * py - ry * px);
}

// W^D = L_p W^s, W^F = (kT / L_p) W^s, blob by blob; W^F is written twice,
// back to back (the right-hand side of both systems of the RFD product).
__global__ __launch_bounds__(kTT) void slip_vectors_kernel(const double* __restrict__ Ws,
                                                          const double* __restrict__ Lp,
                                                          const int* __restrict__ bofs, double kT, int64_t n3,
                                                          double* __restrict__ WD, double* __restrict__ WF) {
    const int b = blockIdx.x;
    const double L = Lp[b], g = kT / Lp[b];
    for (int e = 3 * bofs[b] + threadIdx.x; e < 3 * bofs[b + 1]; e += blockDim.x) {
        WD[e] = L * Ws[e];
        WF[e] = g * Ws[e];
        WF[n3 + e] = g * Ws[e];
    }
}

// D^F_p = ([K^T(Q+) - K^T(Q-)] W^F)_p / delta: force sums and torques about
// the moved tracking points, added over the body's blobs in a fixed order.
__global__ __launch_bounds__(kTT) void force_drift_kernel(const double* __restrict__ posp,
                                                         const double* __restrict__ qp,
                                                         const double* __restrict__ posm,
                                                         const double* __restrict__ qm,
                                                         const double* __restrict__ WF,
                                                         const int* __restrict__ bofs, double inv_delta,
                                                         double* __restrict__ DF) {
    __shared__ double red[6][kTT];
    const int b = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = bofs[b] + threadIdx.x; i < bofs[b + 1]; i += blockDim.x) {
        const double w[3] = {WF[3 * i], WF[3 * i + 1], WF[3 * i + 2]};
        double dp[3], dm[3];
        for (int c = 0; c < 3; ++c) {
            dp[c] = posp[3 * i + c] - qp[3 * b + c];
            dm[c] = posm[3 * i + c] - qm[3 * b + c];
        }
        for (int c = 0; c < 3; ++c) acc[c] += w[c] - w[c];
        acc[3] += (dp[1] * w[2] - dp[2] * w[1]) - (dm[1] * w[2] - dm[2] * w[1]);
        acc[4] += (dp[2] * w[0] - dp[0] * w[2]) - (dm[2] * w[0] - dm[0] * w[2]);
        acc[5] += (dp[0] * w[1] - dp[1] * w[0]) - (dm[0] * w[1] - dm[1] * w[0]);
    }
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int t = 0; t < kTT; ++t) s += red[threadIdx.x][t];
        DF[6 * b + threadIdx.x] = s * inv_delta;
    }
}

// out = ax x + ay y (y may be null; out may be x or y).
__global__ void lincomb_kernel(const double* x, double ax, const double* y, double ay, int64_t n, double* out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = ax * x[e] + (y ? ay * y[e] : 0.0);
}

// EM-T: W^FT_p = kT [W^f_p / L_p, W^tau_p] and dQ_p = [L_p W^f_p, W^tau_p].
__global__ void traction_vectors_kernel(const double* __restrict__ Wf, const double* __restrict__ Wt,
                                        const double* __restrict__ Lp, double kT, int nb, double* __restrict__ WFT,
                                        double* __restrict__ dQ) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    for (int c = 0; c < 3; ++c) {
        WFT[6 * b + c] = kT * Wf[3 * b + c] / Lp[b];
        WFT[6 * b + 3 + c] = kT * Wt[3 * b + c];
        dQ[6 * b + c] = Lp[b] * Wf[3 * b + c];
        dQ[6 * b + 3 + c] = Wt[3 * b + c];
    }
}

// DS_i -= ([K(Q+) - K(Q-)] U)_i / delta = omega_p x ((r+_i - q+_p) - (r-_i - q-_p)) / delta
// (the translational parts cancel).
__global__ __launch_bounds__(kTT) void k_drift_kernel(const double* __restrict__ posp, const double* __restrict__ qp,
                                                     const double* __restrict__ posm, const double* __restrict__ qm,
                                                     const double* __restrict__ U, const int* __restrict__ bofs,
                                                     double inv_delta, double* __restrict__ DS) {
    const int b = blockIdx.x;
    const double wx = U[6 * b + 3], wy = U[6 * b + 4], wz = U[6 * b + 5];
    for (int i = bofs[b] + threadIdx.x; i < bofs[b + 1]; i += blockDim.x) {
        double e[3];
        for (int c = 0; c < 3; ++c) e[c] = (posp[3 * i + c] - qp[3 * b + c]) - (posm[3 * i + c] - qm[3 * b + c]);
        DS[3 * i] -= (wy * e[2] - wz * e[1]) * inv_delta;
        DS[3 * i + 1] -= (wz * e[0] - wx * e[2]) * inv_delta;
        DS[3 * i + 2] -= (wx * e[1] - wy * e[0]) * inv_delta;
    }
}

unsigned gridn(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Bodies {
    int* bofs = nullptr;
    int nb = 0;
};

int upload_bodies(const int64_t* body_offsets, int nb, Arena& ar, hipStream_t st, Bodies& bd) {
    std::vector<int> hb(nb + 1);
    for (int p = 0; p <= nb; ++p) hb[p] = (int)body_offsets[p];
    bd.nb = nb;
    bd.bofs = (int*)ar.take(hb.size() * sizeof(int));
    if (!bd.bofs) return RPYW_ENOMEM;
    return stage_upload(hb.data(), hb.size() * sizeof(int), bd.bofs, st);
}

int lincomb(const double* x, double ax, const double* y, double ay, int64_t n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(lincomb_kernel, dim3(gridn(n)), dim3(256), 0, st, x, ax, y, ay, n, out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

// Keeps the worst status: errors (< 0) win, then not-converged warnings.
void merge(int& rc, int r) {
    if (r < 0 || rc == RPYW_OK) rc = r;
}

}  // namespace

int body_blobs(const double* q, const double* theta, const double* ref, const int* bofs_dev, int nb, double* pos,
               hipStream_t st) {
    hipLaunchKernelGGL(body_blobs_kernel, dim3(nb), dim3(kTT), 0, st, q, theta, ref, bofs_dev, pos);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int body_move(const double* q, const double* theta, const double* U, const double* U2, double h, int nb,
              double* q_out, double* theta_out, hipStream_t st) {
    hipLaunchKernelGGL(body_move_kernel, dim3(gridn(nb)), dim3(256), 0, st, q, theta, U, U2, h, nb, q_out,
                       theta_out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

size_t ts_state_bytes(int64_t N, int nb) {
    return 2 * align_up((size_t)3 * N * sizeof(double)) + 2 * align_up((size_t)6 * nb * sizeof(double));
}

size_t ts_ws_bytes(int64_t N, int max_iter, int nb, int prec) {
    const size_t n3 = (size_t)3 * N;
    size_t b = align_up((size_t)(nb + 1) * sizeof(int));
    // T-S: pos0, W^D, W^F (x2), lambda, pos+-, U+-, slip; EM-T: pos0,
    // lambda (x2), pos+-, U+-, D^S, slip
    b += 10 * align_up(n3 * sizeof(double));
    b += 8 * align_up((size_t)6 * nb * sizeof(double));     // body vectors (q+- counts as one)
    b += 2 * align_up((size_t)4 * nb * sizeof(double));     // theta+-
    b += body_factors_bytes(N, nb) + 2 * kAlign;  // factors shared by the solves at Q^n, and their flag
    size_t sub = rigid_ws_bytes(N, max_iter, nb, prec);
    sub = std::max(sub, lanczos_ws_bytes(N, max_iter, nb, prec));
    sub = std::max(sub, batched_ws_bytes(2 * N, 2, 1, prec));
    sub = std::max(sub, product_ws_bytes(N, prec, 1));
    return b + sub + 16 * kAlign;
}

// Preconditioner factors of one configuration, built once for the solves
// that share it (their flag is checked by each solve).
int shared_factors(const double* pos, int64_t N, double a, double eta, const int64_t* body_offsets, int nb,
                   Arena& ar, hipStream_t st, BodyFactors& pc) {
    int* flag = (int*)ar.take(sizeof(int));
    if (!flag) return RPYW_ENOMEM;
    RPYW_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    return body_factors_build(pos, N, a, eta, body_offsets, nb, ar, st, pc, flag);
}

int ts_predict(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb,
               int64_t N, const double* Lp, const double* FT, const double* Ws, const double* Wn, double kT,
               double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter, int prec,
               double* q_t, double* theta_t, double* pos_t, double* state, Arena& ar, int* iters,
               hipStream_t st) {
    const int64_t n3 = 3 * N;
    Bodies bd;
    int rc = upload_bodies(body_offsets, nb, ar, st, bd);
    if (rc) return rc;
    double* pos0 = (double*)ar.take(n3 * sizeof(double));
    double* WD = (double*)ar.take(n3 * sizeof(double));
    double* WF = (double*)ar.take(2 * n3 * sizeof(double));
    double* lam = (double*)ar.take(n3 * sizeof(double));
    double* pospm = (double*)ar.take(2 * n3 * sizeof(double));
    double* Upm = (double*)ar.take(2 * n3 * sizeof(double));
    double* dQ = (double*)ar.take((size_t)6 * nb * sizeof(double));
    double* qpm = (double*)ar.take((size_t)6 * nb * sizeof(double));
    double* thpm = (double*)ar.take((size_t)8 * nb * sizeof(double));
    if (!pos0 || !WD || !WF || !lam || !pospm || !Upm || !dQ || !qpm || !thpm) return RPYW_ENOMEM;
    double* root = state;                          // c M^{1/2} W^n  [3N]
    double* DS = state + align_up(n3 * 8) / 8;     // [3N]
    double* DF = DS + align_up(n3 * 8) / 8;        // [6 nb]
    double* U0 = DF + align_up((size_t)6 * nb * 8) / 8;  // [6 nb]
    int status = RPYW_OK;
    int it = 0;
    double res = 0.0;

    if ((rc = body_blobs(q, theta, ref, bd.bofs, nb, pos0, st))) return rc;
    hipLaunchKernelGGL(slip_vectors_kernel, dim3(nb), dim3(kTT), 0, st, Ws, Lp, bd.bofs, kT, n3, WD, WF);
    RPYW_HIP(hipGetLastError());
    // one set of preconditioner factors for the three solves at Q^n
    BodyFactors pc0;
    if ((rc = shared_factors(pos0, N, a, eta, body_offsets, nb, ar, st, pc0))) return rc;
    // RFD displacement problem (the sub-solvers keep what they take from the
    // arena, so it is rewound after each)
    const size_t mark = ar.used;
    rc = rigid_solve(pos0, q, body_offsets, nb, WD, nullptr, lam, dQ, N, a, eta, tol, max_iter, prec, ar, &it, &res,
                     st, dom, &pc0);
    ar.used = mark;
    iters[0] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    // Q+- and the drifts
    if ((rc = body_move(q, theta, dQ, nullptr, 0.5 * delta, nb, qpm, thpm, st))) return rc;
    if ((rc = body_move(q, theta, dQ, nullptr, -0.5 * delta, nb, qpm + 3 * nb, thpm + 4 * nb, st))) return rc;
    if ((rc = body_blobs(qpm, thpm, ref, bd.bofs, nb, pospm, st))) return rc;
    if ((rc = body_blobs(qpm + 3 * nb, thpm + 4 * nb, ref, bd.bofs, nb, pospm + n3, st))) return rc;
    hipLaunchKernelGGL(force_drift_kernel, dim3(nb), dim3(kTT), 0, st, pospm, qpm, pospm + n3, qpm + 3 * nb, WF,
                       bd.bofs, 1.0 / delta, DF);
    RPYW_HIP(hipGetLastError());
    if (dom.periodic()) {
        if ((rc = products(pospm, WF, Upm, N, 1, a, eta, prec, ar, st, dom))) return rc;
        if ((rc = products(pospm + n3, WF, Upm + n3, N, 1, a, eta, prec, ar, st, dom))) return rc;
    } else {
        const int64_t so[3] = {0, N, 2 * N};  // Q+ and Q- as two systems of one launch
        if ((rc = batched_products(pospm, so, 2, WF, Upm, 1, a, eta, prec, ar, st))) return rc;
    }
    if ((rc = lincomb(Upm, 1.0 / delta, Upm + n3, -1.0 / delta, n3, DS, st))) return rc;
    // Brownian slip c M^{1/2} W^n
    double err = 0.0;
    rc = lanczos_sqrt(pos0, Wn, lam, N, a, eta, body_offsets, nb, tol, max_iter, prec, ar, &it, &err, st, dom,
                      &pc0);
    ar.used = mark;
    iters[1] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = lincomb(lam, std::sqrt(2.0 * kT / dt), nullptr, 0.0, n3, root, st))) return rc;
    // predictor
    rc = rigid_solve(pos0, q, body_offsets, nb, root, FT, lam, U0, N, a, eta, tol, max_iter, prec, ar, &it, &res, st,
                     dom, &pc0);
    ar.used = mark;
    iters[2] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = body_move(q, theta, U0, nullptr, dt, nb, q_t, theta_t, st))) return rc;
    if ((rc = body_blobs(q_t, theta_t, ref, bd.bofs, nb, pos_t, st))) return rc;
    return status;
}

int ts_correct(const double* q, const double* theta, const double* q_t, const double* theta_t, const double* ref,
               const int64_t* body_offsets, int nb, int64_t N, const double* FT_t, const double* state, double dt,
               double a, double eta, const Domain& dom, double tol, int max_iter, int prec, double* q_next,
               double* theta_next, Arena& ar, int* iters, hipStream_t st) {
    const int64_t n3 = 3 * N;
    Bodies bd;
    int rc = upload_bodies(body_offsets, nb, ar, st, bd);
    if (rc) return rc;
    const double* root = state;
    const double* DS = state + align_up(n3 * 8) / 8;
    const double* DF = DS + align_up(n3 * 8) / 8;
    const double* U0 = DF + align_up((size_t)6 * nb * 8) / 8;
    double* pos_t = (double*)ar.take(n3 * sizeof(double));
    double* slip = (double*)ar.take(n3 * sizeof(double));
    double* lam = (double*)ar.take(n3 * sizeof(double));
    double* F = (double*)ar.take((size_t)6 * nb * sizeof(double));
    double* Ut = (double*)ar.take((size_t)6 * nb * sizeof(double));
    if (!pos_t || !slip || !lam || !F || !Ut) return RPYW_ENOMEM;
    if ((rc = body_blobs(q_t, theta_t, ref, bd.bofs, nb, pos_t, st))) return rc;
    if ((rc = lincomb(DS, 2.0, root, 1.0, n3, slip, st))) return rc;
    if ((rc = lincomb(FT_t, 1.0, DF, -2.0, 6 * (int64_t)nb, F, st))) return rc;
    int it = 0;
    double res = 0.0;
    rc = rigid_solve(pos_t, q_t, body_offsets, nb, slip, F, lam, Ut, N, a, eta, tol, max_iter, prec, ar, &it, &res,
                     st, dom);
    iters[0] = it;
    if (rc < 0) return rc;
    const int status = rc;
    if ((rc = body_move(q, theta, U0, Ut, 0.5 * dt, nb, q_next, theta_next, st))) return rc;
    return status;
}

int emt_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb, int64_t N,
             const double* Lp, const double* FT, const double* Wf, const double* Wt, const double* Wn, double kT,
             double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter, int prec,
             double* q_next, double* theta_next, Arena& ar, int* iters, hipStream_t st) {
    const int64_t n3 = 3 * N, n6 = 6 * (int64_t)nb;
    Bodies bd;
    int rc = upload_bodies(body_offsets, nb, ar, st, bd);
    if (rc) return rc;
    double* pos0 = (double*)ar.take(n3 * sizeof(double));
    double* lam2 = (double*)ar.take(2 * n3 * sizeof(double));  // lambda^RFD twice (both RFD systems)
    double* pospm = (double*)ar.take(2 * n3 * sizeof(double));
    double* Upm = (double*)ar.take(2 * n3 * sizeof(double));
    double* DS = (double*)ar.take(n3 * sizeof(double));
    double* slip = (double*)ar.take(n3 * sizeof(double));
    double* WFT = (double*)ar.take(n6 * sizeof(double));
    double* dQ = (double*)ar.take(n6 * sizeof(double));
    double* Ur = (double*)ar.take(n6 * sizeof(double));
    double* DF = (double*)ar.take(n6 * sizeof(double));
    double* F = (double*)ar.take(n6 * sizeof(double));
    double* U0 = (double*)ar.take(n6 * sizeof(double));
    double* qpm = (double*)ar.take(n6 * sizeof(double));
    double* thpm = (double*)ar.take((size_t)8 * nb * sizeof(double));
    if (!pos0 || !lam2 || !pospm || !Upm || !DS || !slip || !WFT || !dQ || !Ur || !DF || !F || !U0 || !qpm || !thpm)
        return RPYW_ENOMEM;
    int status = RPYW_OK, it = 0;
    double res = 0.0, err = 0.0;
    if ((rc = body_blobs(q, theta, ref, bd.bofs, nb, pos0, st))) return rc;
    hipLaunchKernelGGL(traction_vectors_kernel, dim3(gridn(nb)), dim3(256), 0, st, Wf, Wt, Lp, kT, nb, WFT, dQ);
    RPYW_HIP(hipGetLastError());
    BodyFactors pc0;  // shared by the three solves at Q^n
    if ((rc = shared_factors(pos0, N, a, eta, body_offsets, nb, ar, st, pc0))) return rc;
    // RFD mobility problem: no slip, random force and torque W^FT (the
    // sub-solvers keep what they take from the arena: rewound after each)
    const size_t mark = ar.used;
    rc = rigid_solve(pos0, q, body_offsets, nb, nullptr, WFT, lam2, Ur, N, a, eta, tol, max_iter, prec, ar, &it, &res,
                     st, dom, &pc0);
    ar.used = mark;
    iters[0] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = lincomb(lam2, 1.0, nullptr, 0.0, n3, lam2 + n3, st))) return rc;
    if ((rc = body_move(q, theta, dQ, nullptr, 0.5 * delta, nb, qpm, thpm, st))) return rc;
    if ((rc = body_move(q, theta, dQ, nullptr, -0.5 * delta, nb, qpm + 3 * nb, thpm + 4 * nb, st))) return rc;
    if ((rc = body_blobs(qpm, thpm, ref, bd.bofs, nb, pospm, st))) return rc;
    if ((rc = body_blobs(qpm + 3 * nb, thpm + 4 * nb, ref, bd.bofs, nb, pospm + n3, st))) return rc;
    hipLaunchKernelGGL(force_drift_kernel, dim3(nb), dim3(kTT), 0, st, pospm, qpm, pospm + n3, qpm + 3 * nb, lam2,
                       bd.bofs, 1.0 / delta, DF);
    RPYW_HIP(hipGetLastError());
    if (dom.periodic()) {
        if ((rc = products(pospm, lam2, Upm, N, 1, a, eta, prec, ar, st, dom))) return rc;
        if ((rc = products(pospm + n3, lam2, Upm + n3, N, 1, a, eta, prec, ar, st, dom))) return rc;
    } else {
        const int64_t so[3] = {0, N, 2 * N};
        if ((rc = batched_products(pospm, so, 2, lam2, Upm, 1, a, eta, prec, ar, st))) return rc;
    }
    if ((rc = lincomb(Upm, 1.0 / delta, Upm + n3, -1.0 / delta, n3, DS, st))) return rc;
    hipLaunchKernelGGL(k_drift_kernel, dim3(nb), dim3(kTT), 0, st, pospm, qpm, pospm + n3, qpm + 3 * nb, Ur, bd.bofs,
                       1.0 / delta, DS);
    RPYW_HIP(hipGetLastError());
    // Brownian slip and the mobility problem
    rc = lanczos_sqrt(pos0, Wn, slip, N, a, eta, body_offsets, nb, tol, max_iter, prec, ar, &it, &err, st, dom,
                      &pc0);
    ar.used = mark;
    iters[1] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = lincomb(slip, std::sqrt(2.0 * kT / dt), DS, 1.0, n3, slip, st))) return rc;
    if ((rc = lincomb(FT, 1.0, DF, -1.0, n6, F, st))) return rc;
    rc = rigid_solve(pos0, q, body_offsets, nb, slip, F, lam2, U0, N, a, eta, tol, max_iter, prec, ar, &it, &res, st,
                     dom, &pc0);
    ar.used = mark;
    iters[2] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = body_move(q, theta, U0, nullptr, dt, nb, q_next, theta_next, st))) return rc;
    return status;
}

int emrfd_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb,
               int64_t N, const double* Lp, const double* FT, const double* Wf, const double* Wt, const double* Wn,
               double kT, double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter,
               int prec, double* q_next, double* theta_next, Arena& ar, int* iters, hipStream_t st) {
    const int64_t n3 = 3 * N, n6 = 6 * (int64_t)nb;
    Bodies bd;
    int rc = upload_bodies(body_offsets, nb, ar, st, bd);
    if (rc) return rc;
    double* pos = (double*)ar.take(n3 * sizeof(double));
    double* lam = (double*)ar.take(n3 * sizeof(double));
    double* WFT = (double*)ar.take(n6 * sizeof(double));
    double* dQ = (double*)ar.take(n6 * sizeof(double));
    double* Upm = (double*)ar.take(2 * n6 * sizeof(double));
    double* U0 = (double*)ar.take(n6 * sizeof(double));
    double* qpm = (double*)ar.take(n6 * sizeof(double));
    double* thpm = (double*)ar.take((size_t)8 * nb * sizeof(double));
    if (!pos || !lam || !WFT || !dQ || !Upm || !U0 || !qpm || !thpm) return RPYW_ENOMEM;
    int status = RPYW_OK, it = 0;
    double res = 0.0, err = 0.0;
    hipLaunchKernelGGL(traction_vectors_kernel, dim3(gridn(nb)), dim3(256), 0, st, Wf, Wt, Lp, kT, nb, WFT, dQ);
    RPYW_HIP(hipGetLastError());
    const size_t mark = ar.used;
    // the two RFD mobility problems at Q+ and Q- (no slip, force W^FT)
    for (int sgn = 0; sgn < 2; ++sgn) {
        double* qs = qpm + 3 * nb * sgn;
        double* ts = thpm + 4 * nb * sgn;
        if ((rc = body_move(q, theta, dQ, nullptr, sgn == 0 ? 0.5 * delta : -0.5 * delta, nb, qs, ts, st))) return rc;
        if ((rc = body_blobs(qs, ts, ref, bd.bofs, nb, pos, st))) return rc;
        rc = rigid_solve(pos, qs, body_offsets, nb, nullptr, WFT, lam, Upm + n6 * sgn, N, a, eta, tol, max_iter, prec,
                         ar, &it, &res, st, dom);
        ar.used = mark;
        iters[sgn] = it;
        if (rc < 0) return rc;
        merge(status, rc);
    }
    // Brownian slip and the mobility problem at Q^n (one set of factors)
    if ((rc = body_blobs(q, theta, ref, bd.bofs, nb, pos, st))) return rc;
    BodyFactors pc0;
    if ((rc = shared_factors(pos, N, a, eta, body_offsets, nb, ar, st, pc0))) return rc;
    double* lam0 = (double*)ar.take(n3 * sizeof(double));
    if (!lam0) return RPYW_ENOMEM;
    const size_t mark2 = ar.used;
    rc = lanczos_sqrt(pos, Wn, lam, N, a, eta, body_offsets, nb, tol, max_iter, prec, ar, &it, &err, st, dom, &pc0);
    ar.used = mark2;
    iters[2] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    if ((rc = lincomb(lam, std::sqrt(2.0 * kT / dt), nullptr, 0.0, n3, lam, st))) return rc;
    rc = rigid_solve(pos, q, body_offsets, nb, lam, FT, lam0, U0, N, a, eta, tol, max_iter, prec, ar, &it, &res, st,
                     dom, &pc0);
    ar.used = mark2;
    iters[3] = it;
    if (rc < 0) return rc;
    merge(status, rc);
    // U = U^n + (U+ - U-) / delta, then Q^{n+1} = Q^n + dt U
    if ((rc = lincomb(Upm, 1.0 / delta, Upm + n6, -1.0 / delta, n6, Upm, st))) return rc;
    if ((rc = body_move(q, theta, U0, Upm, dt, nb, q_next, theta_next, st))) return rc;
    return status;
}

}  // namespace rpyw
