// Rigid multiblob mobility problem (arXiv:1709.02410, Sec. II.A): the
// saddle-point system
//
//     [ M   -K ] [lambda]   [-slip]
//     [-K^T  0 ] [  U   ] = [ -F  ]
//
// for blob forces lambda [N][3] and body velocities U = (u_p, omega_p), with
// (K U)_i = u_p + omega_p x (r_i - q_p) for blob i of body p, solved by
// GMRES right-preconditioned with the block-diagonal operator of Sec. II.B:
// interactions between distinct bodies dropped, each body's own block
// M^(pp) kept (wall included), so the preconditioner is the exact inverse
// of one small saddle-point system per body:
//
//     z_U      = -N_p (r_U + W_p^T r_lambda),   W_p = M_pp^-1 K_p,
//     z_lambda = M_pp^-1 r_lambda + W_p z_U,    N_p = (K_p^T W_p)^-1,
//
// with M_pp^-1 = L_p^-T L_p^-1 from the factors the Lanczos solver uses.
// Krylov vectors are [lambda (3N) | U (6 n_bodies)] in FP64; every Arnoldi
// step costs one product by M plus O(N) work.  Classical Gram-Schmidt is
// applied twice; the Hessenberg column goes to pinned host memory, where
// Givens rotations give the residual.  Step k + 1 only needs the norm
// h_{k+1,k} on the device, so for small problems it is queued before the
// host has examined step k (and is discarded if step k converged).
#include <algorithm>
#include <mutex>
#include <cstring>
#include <atomic>
#include <cmath>
#include <vector>

#include "krylov_step.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

constexpr int kRT = 128;  // threads per body (bodies have at most 42 blobs)
constexpr int kMaxN3 = 3 * kMaxBodyBlobs;

// Entry (alpha, col) of the 3 x 6 block of K for a blob at d = r_i - q_p:
// the identity for col < 3 and, for col = 3 + beta, (e_beta x d)_alpha.
__device__ inline double k_entry(int alpha, int col, const double d[3]) {
    if (col < 3) return alpha == col ? 1.0 : 0.0;
    const int beta = col - 3;
    if (alpha == beta) return 0.0;
    const int g = 3 - alpha - beta;                                      // the remaining index
    const double sgn = ((beta - alpha + 3) % 3 == 1) ? 1.0 : -1.0;       // Levi-Civita eps(alpha, beta, g)
    return sgn * d[g];
}

// Sum over j < len of F[j fs] x[j xs] in four partial sums (j = i (mod 4)),
// added pairwise, so that the reads of a step issue together.
__device__ __forceinline__ double dot4s(const double* F, int fs, const double* x, int xs, int len) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 4 <= len; j += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) s4[i] = fma(F[(j + i) * fs], x[(j + i) * xs], s4[i]);
    }
    for (int i = 0; j + i < len; ++i) s4[i] = fma(F[(j + i) * fs], x[(j + i) * xs], s4[i]);
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// Per body: W_p = M_pp^-1 K_p ([3n][6], at 18 bofs[p]) and the 6 x 6 body
// mobility N_p = (K_p^T W_p)^-1 (at 36 p).  Sets *notspd when K_p^T W_p is
// not numerically positive definite (a body whose blobs do not fix all six
// rigid motions, e.g. a single blob or a straight rod).  The inverse factor
// is staged in LDS when it fits (bodies of up to 21 blobs); the 6 x 6
// inverse is a Cholesky factorisation on one thread, then the six columns of
// its inverse factor on six threads and the 36 entries of N on 36.
__global__ __launch_bounds__(kRT) void rigid_factors_kernel(const double* __restrict__ pos,
                                                           const double* __restrict__ q,
                                                           const int* __restrict__ bofs,
                                                           const int64_t* __restrict__ lofs,
                                                           const double* __restrict__ Lall, double* __restrict__ Wall,
                                                           double* __restrict__ Nall, int* __restrict__ notspd) {
    __shared__ double Kl[kMaxN3][6], X[kMaxN3][6], Wl[kMaxN3][6];
    __shared__ double Ls[kstep::kLdsFactor];
    __shared__ double G[6][6], A[6][6], Linv[6][6], rdg[6];
    __shared__ int bad;
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = bofs[p], n = 3 * (bofs[p + 1] - b0);
    const double* Lg = Lall + 2 * lofs[p] + (int64_t)n * n;  // L^-1, row-major
    const bool staged = n * n <= kstep::kLdsFactor;
    kstep::Staged<kRT, kstep::kLdsFactor / kRT> sl;
    if (staged) sl.load(Lg, n * n);
    for (int idx = t; idx < 6 * n; idx += kRT) {
        const int i = idx / 6, c = idx % 6;
        const int blob = b0 + i / 3;
        const double d[3] = {pos[3 * blob] - q[3 * p], pos[3 * blob + 1] - q[3 * p + 1],
                             pos[3 * blob + 2] - q[3 * p + 2]};
        Kl[i][c] = k_entry(i % 3, c, d);
    }
    if (staged) sl.store(Ls, n * n);
    __syncthreads();
    const double* Li = staged ? Ls : Lg;
    for (int idx = t; idx < 6 * n; idx += kRT) {  // X = L^-1 K
        const int i = idx / 6, c = idx % 6;
        X[i][c] = dot4s(Li + (int64_t)i * n, 1, &Kl[0][c], 6, i + 1);
    }
    __syncthreads();
    double* Wp = Wall + 18 * (int64_t)b0;
    for (int idx = t; idx < 6 * n; idx += kRT) {  // W = L^-T X
        const int i = idx / 6, c = idx % 6;
        const double s = dot4s(Li + (int64_t)i * n + i, n, &X[i][c], 6, n - i);
        Wl[i][c] = s;
        Wp[idx] = s;
    }
    __syncthreads();
    if (t < 36) {  // G = K^T W
        const int c = t / 6, e = t % 6;
        double s = 0.0;
        for (int i = 0; i < n; ++i) s = fma(Kl[i][c], Wl[i][e], s);
        G[c][e] = s;
    }
    __syncthreads();
    if (t == 0) {
        // Cholesky of the symmetrised G, with the reciprocals of its diagonal
        double dmax = 0.0;
        for (int i = 0; i < 6; ++i) {
            for (int j = 0; j < 6; ++j) A[i][j] = 0.5 * (G[i][j] + G[j][i]);
            dmax = fmax(dmax, fabs(A[i][i]));
        }
        int b = !(dmax > 0.0);
        for (int k = 0; k < 6 && !b; ++k) {
            double dk = A[k][k];
            for (int m = 0; m < k; ++m) dk -= A[k][m] * A[k][m];
            if (!(dk > 1e-12 * dmax)) {
                b = 1;
                break;
            }
            dk = sqrt(dk);
            A[k][k] = dk;
            rdg[k] = 1.0 / dk;
            for (int i = k + 1; i < 6; ++i) {
                double s = A[i][k];
                for (int m = 0; m < k; ++m) s -= A[i][m] * A[k][m];
                A[i][k] = s * rdg[k];
            }
        }
        bad = b;
        if (b) atomicOr(notspd, 1);
    }
    __syncthreads();
    if (bad) {
        if (t < 36) Nall[36 * (int64_t)p + t] = 0.0;
        return;
    }
    if (t < 6) {  // column t of the inverse factor, by forward substitution
        for (int i = 0; i < 6; ++i) {
            double s = (i == t) ? 1.0 : 0.0;
            for (int m = 0; m < i; ++m) s -= A[i][m] * Linv[m][t];
            Linv[i][t] = s * rdg[i];
        }
    }
    __syncthreads();
    if (t < 36) {  // N = L^-T L^-1
        const int i = t / 6, j = t % 6;
        double s = 0.0;
        for (int m = 0; m < 6; ++m) s = fma(Linv[m][i], Linv[m][j], s);
        Nall[36 * (int64_t)p + t] = s;
    }
}

// z = P^-1 r for r = [rl (3N) | ru (6 nb)] (see the file comment).  With
// scale the input is r / scale[0] and, with store (pointing at a full
// vector), that scaled input is also written there.
// The input r may be the output z (in place): a workgroup reads all of its
// body's input entries before it writes any output, and touches no other
// body's entries.  With nc > 0 the input is first r - sum_{j < nc} c[j] V_j
// (V_j at V + j (n3 + 6 nb), the terms subtracted in order).
__global__ __launch_bounds__(kRT) void rigid_precond_kernel(const double* __restrict__ Lall,
                                                           const int* __restrict__ bofs,
                                                           const int64_t* __restrict__ lofs,
                                                           const double* __restrict__ Wall,
                                                           const double* __restrict__ Nall, int64_t n3,
                                                           const double* rl, const double* ru,
                                                           const double* __restrict__ scale,
                                                           double* __restrict__ store, double* zl, double* zu,
                                                           const double* __restrict__ V, int64_t ld,
                                                           const double* __restrict__ c, int nc) {
    __shared__ double r[kMaxN3], t1[kMaxN3], t[kMaxN3];
    __shared__ double r6[6], s6[6], z6[6];
    const int p = blockIdx.x;
    const int b0 = bofs[p], n = 3 * (bofs[p + 1] - b0);
    const int64_t e0 = 3 * (int64_t)b0;
    const double* Li = Lall + 2 * lofs[p] + (int64_t)n * n;
    const double* W = Wall + 18 * (int64_t)b0;
    const double inv = scale ? 1.0 / scale[0] : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = nc > 0 ? minus_comb(rl, V, ld, c, nc, e0 + i) : rl[e0 + i];
        const double v = scale ? x * inv : x;
        r[i] = v;
        if (store) store[e0 + i] = v;
    }
    if (threadIdx.x < 6) {
        // the U part of V_j starts at n3 (ru = rl + n3 in every call)
        const int64_t eu = 6 * p + threadIdx.x;
        const double x = nc > 0 ? minus_comb(ru, V + n3, ld, c, nc, eu) : ru[eu];
        const double v = scale ? x * inv : x;
        r6[threadIdx.x] = v;
        if (store) store[n3 + eu] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // t1 = L^-1 r
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += Li[(int64_t)i * n + j] * r[j];
        t1[i] = s;
    }
    if (threadIdx.x < 6) {  // s = W^T r = K^T M^-1 r
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += W[6 * i + threadIdx.x] * r[i];
        s6[threadIdx.x] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // t = L^-T t1 = M^-1 r
        double s = 0.0;
        for (int j = i; j < n; ++j) s += Li[(int64_t)j * n + i] * t1[j];
        t[i] = s;
    }
    if (threadIdx.x < 6) {  // z_U = -N (r_U + s)
        const double* Np = Nall + 36 * (int64_t)p + 6 * threadIdx.x;
        double s = 0.0;
        for (int e = 0; e < 6; ++e) s += Np[e] * (r6[e] + s6[e]);
        z6[threadIdx.x] = -s;
        zu[6 * p + threadIdx.x] = -s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // z_lambda = t + W z_U
        double s = t[i];
        for (int c = 0; c < 6; ++c) s += W[6 * i + c] * z6[c];
        zl[e0 + i] = s;
    }
}

// out = A x with x = [xl | xu]: outl = y - K xu (y = M xl already formed),
// outu = -K^T xl.  One workgroup per body.
__global__ __launch_bounds__(kRT) void rigid_apply_kernel(const double* __restrict__ pos,
                                                         const double* __restrict__ q,
                                                         const int* __restrict__ bofs,
                                                         const double* __restrict__ xl,
                                                         const double* __restrict__ xu,
                                                         const double* __restrict__ y, double* __restrict__ outl,
                                                         double* __restrict__ outu) {
    __shared__ double red[6][kMaxBodyBlobs];
    const int p = blockIdx.x;
    const int b0 = bofs[p], nb = bofs[p + 1] - b0;
    for (int a = threadIdx.x; a < nb; a += blockDim.x) {
        const int64_t i = b0 + a;
        const double d[3] = {pos[3 * i] - q[3 * p], pos[3 * i + 1] - q[3 * p + 1], pos[3 * i + 2] - q[3 * p + 2]};
        const double* U = xu + 6 * (int64_t)p;
        const double ku[3] = {U[0] + U[4] * d[2] - U[5] * d[1], U[1] + U[5] * d[0] - U[3] * d[2],
                              U[2] + U[3] * d[1] - U[4] * d[0]};
        const double l[3] = {xl[3 * i], xl[3 * i + 1], xl[3 * i + 2]};
        for (int c = 0; c < 3; ++c) outl[3 * i + c] = y[3 * i + c] - ku[c];
        red[0][a] = l[0];
        red[1][a] = l[1];
        red[2][a] = l[2];
        red[3][a] = d[1] * l[2] - d[2] * l[1];
        red[4][a] = d[2] * l[0] - d[0] * l[2];
        red[5][a] = d[0] * l[1] - d[1] * l[0];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int a = 0; a < nb; ++a) s += red[threadIdx.x][a];
        outu[6 * p + threadIdx.x] = -s;
    }
}

// b = [-slip | -F] (absent terms are zero).
__global__ void rigid_rhs_kernel(const double* __restrict__ slip, const double* __restrict__ FT, int64_t n3,
                                 int64_t n6, double* __restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n3)
        b[e] = slip ? -slip[e] : 0.0;
    else if (e < n3 + n6)
        b[e] = FT ? -FT[e - n3] : 0.0;
}

PinnedSlots g_h;  // Hessenberg columns, one slot per step in flight

// Host side of Arnoldi step k: applies the previous Givens rotations to
// column k of H (h: k + 2 entries), forms rotation k, appends the rotated
// column to R and updates g = Q^T (beta e1).  Returns false when the
// residual estimate |g_{k+1}| / beta (into *res) is not finite; *hk1 is
// h_{k+1,k} as computed.
bool givens_column(std::vector<double>& h, int k, std::vector<std::vector<double>>& R, std::vector<double>& cs,
                   std::vector<double>& sn, std::vector<double>& g, double beta, double* res, double* hk1) {
    for (int j = 0; j < k; ++j) {
        const double t0 = cs[j] * h[j] + sn[j] * h[j + 1];
        h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
        h[j] = t0;
    }
    const double rr = std::hypot(h[k], h[k + 1]);
    const double c = rr > 0.0 ? h[k] / rr : 1.0, s = rr > 0.0 ? h[k + 1] / rr : 0.0;
    cs.push_back(c);
    sn.push_back(s);
    *hk1 = h[k + 1];
    h[k] = rr;
    h.resize(k + 1);
    R.push_back(h);
    g.push_back(-s * g[k]);
    g[k] = c * g[k];
    *res = std::fabs(g[k + 1]) / beta;
    return std::isfinite(*res);
}

// The GMRES coefficients: back substitution R y = g (R stored by columns).
std::vector<double> gmres_coefficients(const std::vector<std::vector<double>>& R, const std::vector<double>& g) {
    const int m = (int)R.size();
    std::vector<double> yv(m);
    for (int i = m - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < m; ++j) s -= R[j][i] * yv[j];
        yv[i] = R[i][i] != 0.0 ? s / R[i][i] : 0.0;
    }
    return yv;
}

// The GMRES solution: back substitution R y = g, then x = P^-1 (V y)
// (precond: the preconditioner applied to a device vector, into the
// caller's outputs).
template <class Precond>
int rigid_finish(const std::vector<std::vector<double>>& R, const std::vector<double>& g, double res,
                 bool converged, int* iters, double* res_out, double* d_y, const double* V, int64_t n, double* tmp,
                 hipStream_t st, Precond precond) {
    const int m = (int)R.size();
    *iters = m;
    *res_out = res;
    const std::vector<double> yv = gmres_coefficients(R, g);
    int rc;
    if ((rc = stage_upload(yv.data(), m * sizeof(double), d_y, st))) return rc;
    if ((rc = vec_comb(V, n, m, d_y, tmp, n, st))) return rc;
    if ((rc = precond(tmp))) return rc;
    return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
}

}  // namespace

size_t rigid_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec) {
    const size_t n3 = (size_t)3 * N, n = n3 + (size_t)6 * n_bodies;
    const size_t m = (size_t)max_iter;
    size_t b = body_factors_bytes(N, n_bodies);
    b += align_up((size_t)18 * N * sizeof(double));          // W_p
    b += align_up((size_t)36 * n_bodies * sizeof(double));   // N_p
    b += align_up((m + 1) * n * sizeof(double));              // V
    b += 3 * align_up(n * sizeof(double));                    // z, w, b
    b += align_up(n3 * sizeof(double));                       // y = M z_lambda
    b += align_up((m + 2) * dot_chunks(n) * sizeof(double));  // dot partials
    b += 4 * align_up((m + 8) * sizeof(double));              // c1, c2, norms, coefficients
    b += align_up(sizeof(unsigned)) + align_up(sizeof(int));  // ticket, notspd
    b += product_ws_bytes(N, prec, 1);
    // fused steps: y', the block partials of both projections, c2 and h
    int m4;
    b += align_up(n * sizeof(double));
    b += align_up((m + 2) * (size_t)std::max(n_bodies, 1) * sizeof(double));
    b += align_up((m + 3) * (size_t)lanczos_gs2_blocks((int64_t)n, &m4) * sizeof(double));
    b += align_up((m + 8) * sizeof(double));
    b += align_up((n / 256 + 2) * sizeof(double));  // partials of |b|^2
    b += align_up(n3 * sizeof(double));             // the summed product (large problems)
    return b + 24 * kAlign;
}

namespace {

// The GMRES solve with fused four-launch Arnoldi steps (rigid_step.hip):
// the same recurrence, preconditioner and host-side Givens rotations as the
// driver below, with the product's records written by the preconditioner
// kernel, the product gathered by the operator kernel, and the Hessenberg
// column of step k published by its last kernel (a flag in pinned memory
// instead of an event between steps).
int rigid_fused(const double* pos, const double* q, const int64_t* body_offsets, int n_bodies, const double* slip,
                const double* FT, double* lam_out, double* U_out, int64_t N, double a, double eta, double tol,
                int max_iter, int prec, Arena& ar, int* iters, double* res_out, hipStream_t st, const Domain& dom,
                const BodyFactors* pre, const SymPlan& sp, int ipw) {
    const int64_t n3 = 3 * N, n6 = 6 * (int64_t)n_bodies, n = n3 + n6;
    *iters = 0;
    *res_out = 0.0;
    int m4;
    const int64_t nblk4 = lanczos_gs2_blocks(n, &m4);
    const int rw = rec_width(prec, 1);
    const int64_t npad = (int64_t)sp.ng * sp.G;
    BodyFactors pc;
    double* Wall = (double*)ar.take((size_t)18 * N * sizeof(double));
    double* Nall = (double*)ar.take((size_t)36 * n_bodies * sizeof(double));
    double* V = (double*)ar.take((size_t)(max_iter + 1) * n * sizeof(double));
    double* zb = (double*)ar.take(n * sizeof(double));  // z = P^-1 v_k
    double* wb = (double*)ar.take(n * sizeof(double));  // w = A z
    double* yb = (double*)ar.take(n * sizeof(double));  // y' = w - V c1
    double* bv = (double*)ar.take(n * sizeof(double));
    const int64_t nrhs = rg_rhs_blocks(n);
    double* sqp = (double*)ar.take((size_t)nrhs * sizeof(double));  // partials of |b|^2
    double* part1 = (double*)ar.take((size_t)(max_iter + 2) * n_bodies * sizeof(double));
    double* part2 = (double*)ar.take((size_t)(max_iter + 3) * nblk4 * sizeof(double));
    double* gc1 = (double*)ar.take((max_iter + 8) * sizeof(double));  // c1 of the last step
    double* d_y = (double*)ar.take((max_iter + 8) * sizeof(double));
    int* notspd = (int*)ar.take(sizeof(int));
    // the factor tables (when the factors are built here) in one block,
    // which the first kernel copies from pinned memory
    TableBlock tb;
    int nmax = 1;
    std::vector<int64_t> hl;
    char* d_tab = nullptr;
    if (pre) {
        pc = *pre;
    } else {
        pc.diag = false;
        pc.nb = n_bodies;
        pc.flag = notspd;
        std::vector<int> hb;
        body_factors_tables(body_offsets, n_bodies, hb, hl, &nmax);
        const size_t o_lofs = tb.add(hl.data(), hl.size() * sizeof(int64_t));
        const size_t o_bofs = tb.add(hb.data(), hb.size() * sizeof(int));
        tb.host.resize(align_up(tb.host.size()), 0);
        d_tab = (char*)ar.take(tb.host.size());
        pc.L = (double*)ar.take((size_t)2 * hl[n_bodies] * sizeof(double));
        if (!d_tab || !pc.L) return RPYW_ENOMEM;
        pc.lofs = (int64_t*)(d_tab + o_lofs);
        pc.bofs = (int*)(d_tab + o_bofs);
    }
    const size_t tbytes = tb.host.size();
    void* rec = ar.take((size_t)npad * rw * real_size(prec));
    double* B = (double*)ar.take((size_t)npad * sizeof(double));
    double* tpart = (double*)ar.take(sp.tpart_bytes);
    void* spart = ar.take(sp.spart_bytes);
    double* ypre = krylov_presum(sp) ? (double*)ar.take((size_t)n3 * sizeof(double)) : nullptr;
    if (!Wall || !Nall || !V || !zb || !wb || !yb || !bv || !sqp || !part1 || !part2 || !gc1 || !d_y || !notspd ||
        !rec || !B || !tpart || !spart || (krylov_presum(sp) && !ypre))
        return RPYW_ENOMEM;
    std::lock_guard<std::mutex> lk(g_h.mu);
    const int slot = 2 * (max_iter + 2);  // c1[0..k], c2[0..k], h_{k+1,k}
    const size_t hdr_bytes = align_up(((size_t)PinnedSlots::kSlots * slot + 2 + (max_iter + 2)) * sizeof(double));
    int rc = g_h.reserve(hdr_bytes + tbytes);
    if (rc) return rc;
    SlotRelease slots_done{g_h, st};
    double* h_slot = g_h.p;
    // the header (|b|, then the two definiteness flags), written by pre of
    // step 0 and read by the host with step 0
    double* h_b = h_slot + (size_t)PinnedSlots::kSlots * slot;
    int* h_bad = (int*)(h_b + 1);
    double* dh_hdr = g_h.dp + (h_b - h_slot);
    double* h_flag = h_b + 2;
    double* dh_flag = g_h.dp + (h_flag - h_slot);
    std::memset(h_flag, 0, (size_t)(max_iter + 2) * sizeof(double));
    if (tbytes) std::memcpy((char*)h_slot + hdr_bytes, tb.host.data(), tbytes);
    const int* dh_tab = (const int*)((const char*)g_h.dp + hdr_bytes);

    // b, the partials of |b|^2, the records' positions and B (the force
    // slots are rewritten by every step), the tables, and notspd cleared
    // before the factor kernels
    if ((rc = rg_launch_rhs(prec, pos, N, npad, rw, a, dom, rec, B, slip, FT, n3, n6, bv, sqp, notspd, dh_tab,
                            (int*)d_tab, (int)(tbytes / sizeof(int)), st)))
        return rc;
    if (!pre && (rc = body_factors_launch(pos, N, a, eta, pc, nmax, notspd, st))) return rc;
    hipLaunchKernelGGL(rigid_factors_kernel, dim3(n_bodies), dim3(kRT), 0, st, pos, q, pc.bofs, pc.lofs, pc.L, Wall,
                       Nall, notspd);
    RPYW_HIP(hipGetLastError());
    const double m0 = 1.0 / (6.0 * M_PI * eta * a);

    // Step k: the product of z (records written by pre of step k), w = A z
    // with the first projection, y' = w - V c1 with the second projection,
    // then pre of step k + 1, which publishes the column of step k.
    auto pre_k = [&](int k) {
        return rg_launch_pre(prec, pc, Wall, Nall, n_bodies, n3, n, k ? yb : bv, k ? part2 : sqp,
                             k ? (int)nblk4 : (int)nrhs, gc1, g_h.dp, slot, dh_flag, k, V, zb, zb + n3, rec, rw, B,
                             dh_hdr, notspd, pre ? pre->flag : nullptr, st);
    };
    auto launch_step = [&](int k) -> int {
        int r;
        if ((r = sym_launch(rec, sp, ipw, 1, prec, a, dom, tpart, spart, st))) return r;
        if (ypre && (r = sym_finish(tpart, spart, B, N, 1, 1, prec, sp, m0, ypre, st, nullptr, 1.0 / a))) return r;
        if ((r = rg_launch_out(prec, pos, q, pc.bofs, n_bodies, tpart, spart, sp, B, m0, zb, zb + n3, n3, n, V, k, wb,
                               part1, ypre, st)))
            return r;
        if ((r = lz_launch_gs2(wb, yb, n, V, k, part1, n_bodies, part2, nullptr, gc1, st))) return r;
        if ((r = pre_k(k + 1))) return r;  // V has room for max_iter + 1 vectors
        return RPYW_OK;
    };
    const int depth = (double)N * (double)N <= kSpeculatePairs ? kSpeculateDepth : 0;
    int queued = 0;
    auto fill = [&](int upto) -> int {  // queue steps up to index upto - 1
        for (; queued < upto && queued < max_iter; ++queued)
            if (int r = launch_step(queued)) return r;
        return RPYW_OK;
    };
    // Waits for step k: its flag, polled; the stream is queried now and then
    // so that a stream that drains without setting it ends the wait.
    auto wait_step = [&](int k) -> int {
        const volatile double* f = h_flag + k;
        for (unsigned spin = 1;; ++spin) {
            if (*f != 0.0) break;
            if ((spin & 4095) == 0) {
                const hipError_t qs = hipStreamQuery(st);
                if (qs == hipSuccess) {
                    if (*f != 0.0) break;
                    return RPYW_EHIP;
                }
                if (qs != hipErrorNotReady) return RPYW_EHIP;
            }
            __builtin_ia32_pause();
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        return RPYW_OK;
    };

    std::vector<std::vector<double>> R;
    std::vector<double> cs, sn, g;
    bool converged = false;
    double beta = 0.0, res = 1.0, res1 = INFINITY, res2 = INFINITY;
    int k = 0;
    if ((rc = pre_k(0))) return rc;
    if ((rc = fill(1 + depth))) return rc;
    for (; k < max_iter; ++k) {
        if ((rc = wait_step(k))) return rc;
        if (k == 0) {
            beta = *h_b;
            const bool bad = h_bad[0] || h_bad[1];
            if (bad || !std::isfinite(beta) || beta == 0.0) {
                RPYW_HIP(hipStreamSynchronize(st));
                if (bad) return RPYW_ENOTSPD;
                if (!std::isfinite(beta)) return RPYW_EINVAL;
                RPYW_HIP(hipMemsetAsync(lam_out, 0, n3 * sizeof(double), st));
                RPYW_HIP(hipMemsetAsync(U_out, 0, n6 * sizeof(double), st));
                return RPYW_OK;
            }
            g.assign(1, beta);
        }
        const double* hs = h_slot + (size_t)(k % PinnedSlots::kSlots) * slot;
        std::vector<double> h(k + 2);
        for (int j = 0; j <= k; ++j) h[j] = hs[j] + hs[k + 1 + j];
        h[k + 1] = hs[2 * (k + 1)];
        if (depth && (rc = fill(speculate_to(k, depth, res1, res2, tol) + 1))) return rc;
        double hk1;
        if (!givens_column(h, k, R, cs, sn, g, beta, &res, &hk1)) return RPYW_EHIP;
        if (res <= tol || hk1 <= 1e-14 * beta) {
            converged = true;
            break;
        }
        res2 = res1;
        res1 = res;
        if ((rc = fill(k + 2))) return rc;
    }
    if ((int)R.size() <= kLanczosCoefArgs) {
        // x = P^-1 (V y) in one launch, y passed by value
        const std::vector<double> yv = gmres_coefficients(R, g);
        *iters = (int)R.size();
        *res_out = res;
        if ((rc = rg_launch_fin(pc, Wall, Nall, n_bodies, n3, n, V, yv.data(), (int)yv.size(), lam_out, U_out, st)))
            return rc;
        return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
    }
    return rigid_finish(R, g, res, converged, iters, res_out, d_y, V, n, wb, st, [&](const double* in) {
        hipLaunchKernelGGL(rigid_precond_kernel, dim3(n_bodies), dim3(kRT), 0, st, pc.L, pc.bofs, pc.lofs, Wall, Nall,
                           n3, in, in + n3, nullptr, nullptr, lam_out, U_out, V, n, nullptr, 0);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    });
}

}  // namespace

int rigid_solve(const double* pos, const double* q, const int64_t* body_offsets, int n_bodies, const double* slip,
                const double* FT, double* lam_out, double* U_out, int64_t N, double a, double eta, double tol,
                int max_iter, int prec, Arena& ar, int* iters, double* res_out, hipStream_t st, const Domain& dom,
                const BodyFactors* pre) {
    {
        SymPlan sp;
        int ipw;
        if (n_bodies > 0 && lanczos_fused_applies(N, prec, max_iter, dom, &sp, &ipw))
            return rigid_fused(pos, q, body_offsets, n_bodies, slip, FT, lam_out, U_out, N, a, eta, tol, max_iter,
                               prec, ar, iters, res_out, st, dom, pre, sp, ipw);
    }
    const int64_t n3 = 3 * N, n6 = 6 * (int64_t)n_bodies, n = n3 + n6;
    *iters = 0;
    *res_out = 0.0;
    BodyFactors pc;
    double* Wall = (double*)ar.take((size_t)18 * N * sizeof(double));
    double* Nall = (double*)ar.take((size_t)36 * n_bodies * sizeof(double));
    double* V = (double*)ar.take((size_t)(max_iter + 1) * n * sizeof(double));
    double* z = (double*)ar.take(n * sizeof(double));
    double* w = (double*)ar.take(n * sizeof(double));
    double* bv = (double*)ar.take(n * sizeof(double));
    double* y = (double*)ar.take(n3 * sizeof(double));
    double* partial = (double*)ar.take((size_t)(max_iter + 2) * dot_chunks(n) * sizeof(double));
    // column of step k: c1[0..k], c2[0..k], h_{k+1,k} (one copy to the host)
    double* d_col = (double*)ar.take((2 * max_iter + 8) * sizeof(double));
    double* d_hn = (double*)ar.take((max_iter + 8) * sizeof(double));  // [0] = |b|, [k + 1] = h_{k+1,k}
    double* d_y = (double*)ar.take((max_iter + 8) * sizeof(double));
    unsigned* ticket = (unsigned*)ar.take(kAlign);
    int* notspd = (int*)ar.take(sizeof(int));
    if (!Wall || !Nall || !V || !z || !w || !bv || !y || !partial || !d_col || !d_hn || !d_y || !ticket || !notspd)
        return RPYW_ENOMEM;
    std::lock_guard<std::mutex> lk(g_h.mu);
    const int slot = 2 * (max_iter + 2);  // c1[0..k], c2[0..k], h_{k+1,k}
    int rc = g_h.reserve(((size_t)PinnedSlots::kSlots * slot + 2) * sizeof(double));
    if (rc) return rc;
    SlotRelease slots_done{g_h, st};
    double* h_slot = g_h.p;
    // |b| and the not-positive-definite flags come back with step 0
    double* h_b = h_slot + (size_t)PinnedSlots::kSlots * slot;
    int* h_bad = (int*)(h_b + 1);

    RPYW_HIP(hipMemsetAsync(notspd, 0, sizeof(int), st));
    RPYW_HIP(hipMemsetAsync(ticket, 0, sizeof(unsigned), st));
    if (pre)
        pc = *pre;
    else if ((rc = body_factors_build(pos, N, a, eta, body_offsets, n_bodies, ar, st, pc, notspd)))
        return rc;
    hipLaunchKernelGGL(rigid_factors_kernel, dim3(n_bodies), dim3(kRT), 0, st, pos, q, pc.bofs, pc.lofs, pc.L, Wall,
                       Nall, notspd);
    RPYW_HIP(hipGetLastError());
    hipLaunchKernelGGL(rigid_rhs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, slip, FT, n3, n6, bv);
    RPYW_HIP(hipGetLastError());

    auto precond = [&](const double* in, const double* scale, double* store, double* outl, double* outu,
                       const double* c = nullptr, int nc = 0) -> int {
        hipLaunchKernelGGL(rigid_precond_kernel, dim3(n_bodies), dim3(kRT), 0, st, pc.L, pc.bofs, pc.lofs, Wall, Nall,
                           n3, in, in + n3, scale, store, outl, outu, V, n, c, nc);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    };
    auto dots = [&](const double* vec, int nv, double* res, int copy_idx, double* copy_to) {
        return vec_dots(V, n, nv, vec, n, partial, ticket, res, copy_idx, copy_to, st);
    };

    // beta = |b|
    if ((rc = dots(bv, 0, d_hn, 0, nullptr))) return rc;
    h_bad[0] = h_bad[1] = 0;
    RPYW_HIP(hipMemcpyAsync(h_b, d_hn, sizeof(double), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipMemcpyAsync(h_bad, notspd, sizeof(int), hipMemcpyDeviceToHost, st));
    if (pre && pre->flag) RPYW_HIP(hipMemcpyAsync(h_bad + 1, pre->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    double beta = 0.0;

    // Arnoldi step k: v_k = (k ? z - V c2 : b) / d_hn[k] (the second
    // correction of step k - 1), z = P^-1 v_k, w = A z, then classical
    // Gram-Schmidt twice: c1 = V^T w; z = w - V c1 with c2 = V^T z and |z|^2
    // in the same pass, h_{k+1,k} = |z - V c2| from |z|^2 - |c2|^2 (V
    // orthonormal) into d_hn[k + 1]; column k of H (c1, c2, h) is stored
    // into its pinned slot by that pass.
    auto launch_step = [&](int k) -> int {
        double* vk = V + (size_t)k * n;
        int r;
        if (k == 0)
            r = precond(bv, d_hn, vk, z, z + n3);
        else  // in place: z -> z
            r = precond(z, d_hn + k, vk, z, z + n3, d_col + k, k);
        if (r) return r;
        if ((r = products(pos, z, y, N, 1, a, eta, prec, ar, st, dom))) return r;
        hipLaunchKernelGGL(rigid_apply_kernel, dim3(n_bodies), dim3(kRT), 0, st, pos, q, pc.bofs, z, z + n3, y, w,
                           w + n3);
        RPYW_HIP(hipGetLastError());
        double* c1 = d_col;
        double* c2 = d_col + (k + 1);
        if ((r = dots(w, k + 1, c1, 0, nullptr))) return r;
        double* hs = g_h.dp + (size_t)(k % PinnedSlots::kSlots) * slot;
        if ((r = vec_update_dots(w, z, n, nullptr, nullptr, V, n, c1, k + 1, k + 1, partial, ticket, c2, 0,
                                 d_hn + k + 1, st, hs, d_col, 2 * (k + 1) + 1, true, c2 + (k + 1))))
            return r;
        RPYW_HIP(hipEventRecord(g_h.ev[k % PinnedSlots::kSlots], st));
        return RPYW_OK;
    };
    const int depth = (double)N * (double)N <= kSpeculatePairs ? kSpeculateDepth : 0;
    int queued = 0;
    auto fill = [&](int upto) -> int {  // queue steps up to index upto - 1
        for (; queued < upto && queued < max_iter; ++queued)
            if (int r = launch_step(queued)) return r;
        return RPYW_OK;
    };

    // Host: upper-triangular R (columns), Givens rotations, g = beta e1.
    std::vector<std::vector<double>> R;
    std::vector<double> cs, sn, g;
    bool converged = false;
    double res = 1.0, res1 = INFINITY, res2 = INFINITY;  // residual estimates of steps k - 1, k - 2
    int k = 0;
    if ((rc = fill(1 + depth))) return rc;
    for (; k < max_iter; ++k) {
        RPYW_HIP(hipEventSynchronize(g_h.ev[k % PinnedSlots::kSlots]));
        if (k == 0) {  // the first wait also brings |b| and the flags
            beta = *h_b;
            const bool bad = h_bad[0] || h_bad[1];
            if (bad || !std::isfinite(beta) || beta == 0.0) {
                RPYW_HIP(hipStreamSynchronize(st));  // drain the queued steps
                if (bad) return RPYW_ENOTSPD;
                if (!std::isfinite(beta)) return RPYW_EINVAL;
                RPYW_HIP(hipMemsetAsync(lam_out, 0, n3 * sizeof(double), st));
                RPYW_HIP(hipMemsetAsync(U_out, 0, n6 * sizeof(double), st));
                return RPYW_OK;
            }
            g.assign(1, beta);
        }
        const double* hs = h_slot + (size_t)(k % PinnedSlots::kSlots) * slot;
        std::vector<double> h(k + 2);
        for (int j = 0; j <= k; ++j) h[j] = hs[j] + hs[k + 1 + j];
        h[k + 1] = hs[2 * (k + 1)];
        if (depth && (rc = fill(speculate_to(k, depth, res1, res2, tol) + 1))) return rc;
        double hk1;
        if (!givens_column(h, k, R, cs, sn, g, beta, &res, &hk1)) return RPYW_EHIP;
        if (res <= tol || hk1 <= 1e-14 * beta) {
            converged = true;
            break;
        }
        res2 = res1;
        res1 = res;
        if ((rc = fill(k + 2))) return rc;  // step k + 1, unless queued already
    }
    return rigid_finish(R, g, res, converged, iters, res_out, d_y, V, n, w, st,
                        [&](const double* in) { return precond(in, nullptr, nullptr, lam_out, U_out); });
}

}  // namespace rpyw
