// Preconditioned Lanczos for Brownian blob displacements M^{1/2} W
// (arXiv:1709.02410, Sec. II.B).
//
//   L     block diagonal, one lower Cholesky factor per body of the dense
//         block M^(pp) of that body alone (other bodies ignored, wall kept);
//         built once per call (Sec. II.B, block-diagonal preconditioner).
//   G     = L^-1 M L^-T, applied as L^-T -> product by M -> L^-1.
//   Krylov basis V (FP64, [iter][3N]), three-term recurrence with full
//   reorthogonalisation (two classical Gram-Schmidt passes), alpha/beta kept
//   on the device; one device->host copy of (alpha_k, beta_k) per iteration.
//   Host: eigendecomposition of the k x k tridiagonal T_k, coefficients
//   c_k = beta0 Q Lambda^{1/2} Q^T e1; since V is orthonormal the stopping
//   test |y_k - y_{k-1}| <= tol |y_k| is evaluated on c.  At the end
//   out = L (V c).
// All reductions are two-stage with a fixed order (bitwise reproducible).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pair_math.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

constexpr int kRedBlocks = 512;  // first-stage reduction blocks
constexpr int kBodyThreads = 128;

// Dense M^(pp) of one body (units: physical, includes mu0 and B factors)
// assembled in LDS, then factorised in place (right-looking Cholesky).
__global__ __launch_bounds__(kBodyThreads) void precond_build_kernel(const double* __restrict__ pos,
                                                                     const int* __restrict__ bofs,
                                                                     const int64_t* __restrict__ lofs, double inv_a,
                                                                     double mu0, double* __restrict__ Lout,
                                                                     int* __restrict__ notspd) {
    __shared__ double A[3 * kMaxBodyBlobs][3 * kMaxBodyBlobs + 1];
    __shared__ double px[kMaxBodyBlobs], py[kMaxBodyBlobs], pz[kMaxBodyBlobs], pb[kMaxBodyBlobs];
    __shared__ int bad;
    const int p = blockIdx.x;
    const int b0 = bofs[p], nb = bofs[p + 1] - b0, n = 3 * nb;
    if (threadIdx.x == 0) bad = 0;
    for (int a = threadIdx.x; a < nb; a += blockDim.x) {
        const double x = pos[3 * (b0 + a)] * inv_a, y = pos[3 * (b0 + a) + 1] * inv_a,
                     z = pos[3 * (b0 + a) + 2] * inv_a;
        px[a] = x;
        py[a] = y;
        pz[a] = z < 1.0 ? 1.0 : z;
        pb[a] = z < 1.0 ? z : 1.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) {
        const int ia = q / nb, ib = q % nb;
        const double dx = px[ia] - px[ib], dy = py[ia] - py[ib], dz = pz[ia] - pz[ib];
        const PairCoef<double> c = pair_coef<double>(dx, dy, dz, pz[ia], pz[ib]);
        const double sc = mu0 * pb[ia] * pb[ib];
        for (int beta = 0; beta < 3; ++beta) {
            double u[3] = {0.0, 0.0, 0.0};
            pair_apply<double>(c, dx, dy, dz, beta == 0 ? 1.0 : 0.0, beta == 1 ? 1.0 : 0.0, beta == 2 ? 1.0 : 0.0,
                               u[0], u[1], u[2]);
            for (int al = 0; al < 3; ++al) A[3 * ia + al][3 * ib + beta] = sc * u[al];
        }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) {
            const double d = A[k][k];
            if (!(d > 0.0)) bad = 1;
            A[k][k] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double dk = A[k][k];
        for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i][k] /= dk;
        __syncthreads();
        const int m = n - k - 1;
        for (int q = threadIdx.x; q < m * m; q += blockDim.x) {
            const int i = k + 1 + q / m, j = k + 1 + q % m;
            if (j <= i) A[i][j] -= A[i][k] * A[j][k];
        }
        __syncthreads();
    }
    double* L = Lout + lofs[p];
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int i = q / n, j = q % n;
        L[q] = j <= i ? A[i][j] : 0.0;
    }
    if (threadIdx.x == 0 && bad) atomicOr(notspd, 1);
}

// mode 0: out = L v;  1: out = L^-1 v;  2: out = L^-T v.  One workgroup per
// body; substitution with the segment held in LDS.
__global__ __launch_bounds__(kBodyThreads) void precond_apply_kernel(const double* __restrict__ Lall,
                                                                     const int* __restrict__ bofs,
                                                                     const int64_t* __restrict__ lofs, int mode,
                                                                     const double* __restrict__ v,
                                                                     double* __restrict__ out) {
    __shared__ double x[3 * kMaxBodyBlobs];
    const int p = blockIdx.x;
    const int e0 = 3 * bofs[p], n = 3 * bofs[p + 1] - e0;
    const double* L = Lall + lofs[p];
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = v[e0 + i];
    __syncthreads();
    if (mode == 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double s = 0.0;
            for (int j = 0; j <= i; ++j) s += L[i * n + j] * x[j];
            out[e0 + i] = s;
        }
        return;
    }
    if (mode == 1) {
        for (int k = 0; k < n; ++k) {
            const double xk = x[k] / L[k * n + k];
            __syncthreads();
            if (threadIdx.x == 0) x[k] = xk;
            for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) x[i] -= L[i * n + k] * xk;
            __syncthreads();
        }
    } else {
        for (int k = n - 1; k >= 0; --k) {
            const double xk = x[k] / L[k * n + k];
            __syncthreads();
            if (threadIdx.x == 0) x[k] = xk;
            for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] -= L[k * n + i] * xk;
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[e0 + i] = x[i];
}

// Per-blob 3x3 blocks (no body structure): the self block is diagonal,
// B^2 mu0 diag(mu_par, mu_par, mu_perp), so L is its square root.
__global__ void blob_diag_kernel(const double* __restrict__ pos, int64_t N, double inv_a, double mu0,
                                 double* __restrict__ ldiag, int* __restrict__ notspd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double z = pos[3 * i + 2] * inv_a;
    const double zt = z < 1.0 ? 1.0 : z, B = z < 1.0 ? z : 1.0;
    const PairCoef<double> c = pair_coef<double>(0.0, 0.0, 0.0, zt, zt);
    double u[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    pair_apply<double>(c, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, u[0], u[1], u[2]);
    pair_apply<double>(c, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, w[0], w[1], w[2]);
    const double d[3] = {mu0 * B * B * u[0], mu0 * B * B * u[0], mu0 * B * B * w[2]};
    for (int c2 = 0; c2 < 3; ++c2) {
        if (!(d[c2] > 0.0)) atomicOr(notspd, 1);
        ldiag[3 * i + c2] = d[c2] > 0.0 ? sqrt(d[c2]) : 1.0;
    }
}

// mode 0: out = D v; 1, 2: out = v / D (diagonal L).
__global__ void diag_apply_kernel(const double* __restrict__ ldiag, int64_t n3, int mode, const double* __restrict__ v,
                                  double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    out[e] = mode == 0 ? ldiag[e] * v[e] : v[e] / ldiag[e];
}

// partial[j][blk] = sum over this block's entries of V_j . w, j < nv.
// V_j = V + j * ld.  blockDim = 256.
__global__ __launch_bounds__(256) void dots_partial_kernel(const double* __restrict__ V, int64_t ld, int nv,
                                                           const double* __restrict__ w, int64_t n3,
                                                           double* __restrict__ partial) {
    __shared__ double red[256];
    for (int j = 0; j < nv; ++j) {
        double s = 0.0;
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n3; e += (int64_t)gridDim.x * 256)
            s += V[j * ld + e] * w[e];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[j] = sum_blk partial[j][blk] (fixed order), one block per j.
// If sqrt_out, out[j] = sqrt(sum).
__global__ __launch_bounds__(256) void dots_final_kernel(const double* __restrict__ partial, int nblk,
                                                         double* __restrict__ out, int sqrt_out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)j * nblk + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sqrt_out ? sqrt(red[0]) : red[0];
}

// w -= sum_{j < nv} c[j] V_j
__global__ void sub_vc_kernel(const double* __restrict__ V, int64_t ld, int nv, const double* __restrict__ c,
                              double* __restrict__ w, int64_t n3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    double s = w[e];
    for (int j = 0; j < nv; ++j) s -= c[j] * V[j * ld + e];
    w[e] = s;
}

// out = sum_{j < nv} c[j] V_j
__global__ void vc_kernel(const double* __restrict__ V, int64_t ld, int nv, const double* __restrict__ c,
                          double* __restrict__ out, int64_t n3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += c[j] * V[j * ld + e];
    out[e] = s;
}

// w -= beta * vprev
__global__ void axpy_beta_kernel(const double* __restrict__ beta, const double* __restrict__ vprev,
                                 double* __restrict__ w, int64_t n3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    w[e] -= beta[0] * vprev[e];
}

// out = v / s[0]
__global__ void scale_div_kernel(const double* __restrict__ s, const double* __restrict__ v, double* __restrict__ out,
                                 int64_t n3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    out[e] = v[e] / s[0];
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Precond {
    bool diag = true;
    int nb = 0;
    int* bofs = nullptr;
    int64_t* lofs = nullptr;
    double* L = nullptr;  // factors (bodies) or diagonal [3N]

    int apply(int mode, const double* v, double* out, int64_t n3, hipStream_t st) const {
        if (diag)
            hipLaunchKernelGGL(diag_apply_kernel, dim3(grid_of(n3)), dim3(256), 0, st, L, n3, mode, v, out);
        else
            hipLaunchKernelGGL(precond_apply_kernel, dim3(nb), dim3(kBodyThreads), 0, st, L, bofs, lofs, mode, v, out);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    }
};

}  // namespace

// ---------------------------------------------------- tridiagonal (host)

// Implicit symmetric QL with Wilkinson shifts on T = tridiag(e, d, e);
// accumulates the eigenvectors in Z (row-major k x k, Z[i*k+m] = component i
// of eigenvector m).  Returns false if an eigenvalue needs more than 60
// sweeps.
static bool tridiag_ql(std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z, int k) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Z[i * k + j] = i == j ? 1.0 : 0.0;
    if (k == 1) return true;
    e.resize(k);
    e[k - 1] = 0.0;
    for (int l = 0; l < k; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < k - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            // Wilkinson-type shift from the leading 2x2 block at l.
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int row = 0; row < k; ++row) {
                    f = Z[row * k + i + 1];
                    Z[row * k + i + 1] = s * Z[row * k + i] + c * f;
                    Z[row * k + i] = c * Z[row * k + i] - s * f;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

int tridiag_sqrt_coeffs(const double* alpha, const double* beta, int k, double beta0, double* c) {
    std::vector<double> d(alpha, alpha + k), e(k, 0.0), Z((size_t)k * k);
    for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
    if (!tridiag_ql(d, e, Z, k)) return RPYW_NOT_CONVERGED;
    for (int i = 0; i < k; ++i) {
        double s = 0.0;
        for (int m = 0; m < k; ++m) s += Z[i * k + m] * std::sqrt(std::max(d[m], 0.0)) * Z[m];
        c[i] = beta0 * s;
    }
    return RPYW_OK;
}

// ---------------------------------------------------- driver

size_t lanczos_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec) {
    const size_t n3 = (size_t)3 * N;
    size_t b = 0;
    b += align_up((size_t)(n_bodies + 1) * sizeof(int));
    b += align_up((size_t)(n_bodies + 1) * sizeof(int64_t));
    const size_t lsz = n_bodies > 0 ? (size_t)9 * std::min<int64_t>(N, kMaxBodyBlobs) * N : n3;
    b += align_up(lsz * sizeof(double));
    b += align_up((size_t)(max_iter + 1) * n3 * sizeof(double));  // V
    b += 3 * align_up(n3 * sizeof(double));                        // x, y, w
    b += align_up((size_t)(max_iter + 2) * kRedBlocks * sizeof(double));
    b += 4 * align_up((size_t)(max_iter + 8) * sizeof(double));  // alpha, beta, c, tmp
    b += align_up(sizeof(int));
    b += product_ws_bytes(N, prec, 1);
    return b + 16 * kAlign;
}

int lanczos_sqrt(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                 const int64_t* body_offsets, int n_bodies, double tol, int max_iter, int prec, Arena& ar, int* iters,
                 double* err, hipStream_t st) {
    const int64_t n3 = 3 * N;
    const double inv_a = 1.0 / a, m0 = 1.0 / (6.0 * M_PI * eta * a);
    *iters = 0;
    *err = 0.0;
    Precond pc;
    pc.diag = n_bodies == 0;
    pc.nb = n_bodies;
    int* notspd = nullptr;
    if (!pc.diag) {
        std::vector<int> hb(n_bodies + 1);
        std::vector<int64_t> hl(n_bodies + 1, 0);
        for (int p = 0; p <= n_bodies; ++p) hb[p] = (int)body_offsets[p];
        for (int p = 0; p < n_bodies; ++p) {
            const int64_t n = 3 * (body_offsets[p + 1] - body_offsets[p]);
            hl[p + 1] = hl[p] + n * n;
        }
        pc.bofs = (int*)ar.take(hb.size() * sizeof(int));
        pc.lofs = (int64_t*)ar.take(hl.size() * sizeof(int64_t));
        pc.L = (double*)ar.take((size_t)hl[n_bodies] * sizeof(double));
        if (!pc.bofs || !pc.lofs || !pc.L) return RPYW_ENOMEM;
        RPYW_HIP(hipMemcpyAsync(pc.bofs, hb.data(), hb.size() * sizeof(int), hipMemcpyHostToDevice, st));
        RPYW_HIP(hipMemcpyAsync(pc.lofs, hl.data(), hl.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        RPYW_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
    } else {
        pc.L = (double*)ar.take((size_t)n3 * sizeof(double));
        if (!pc.L) return RPYW_ENOMEM;
    }
    double* V = (double*)ar.take((size_t)(max_iter + 1) * n3 * sizeof(double));
    double* x = (double*)ar.take(n3 * sizeof(double));
    double* y = (double*)ar.take(n3 * sizeof(double));
    double* w = (double*)ar.take(n3 * sizeof(double));
    double* partial = (double*)ar.take((size_t)(max_iter + 2) * kRedBlocks * sizeof(double));
    double* d_alpha = (double*)ar.take((max_iter + 8) * sizeof(double));
    double* d_beta = (double*)ar.take((max_iter + 8) * sizeof(double));
    double* d_c = (double*)ar.take((max_iter + 8) * sizeof(double));
    double* d_tmp = (double*)ar.take((max_iter + 8) * sizeof(double));
    notspd = (int*)ar.take(sizeof(int));
    if (!V || !x || !y || !w || !partial || !d_alpha || !d_beta || !d_c || !d_tmp || !notspd) return RPYW_ENOMEM;
    RPYW_HIP(hipMemsetAsync(notspd, 0, sizeof(int), st));
    if (pc.diag)
        hipLaunchKernelGGL(blob_diag_kernel, dim3(grid_of(N)), dim3(256), 0, st, pos, N, inv_a, m0, pc.L, notspd);
    else
        hipLaunchKernelGGL(precond_build_kernel, dim3(n_bodies), dim3(kBodyThreads), 0, st, pos, pc.bofs, pc.lofs,
                           inv_a, m0, pc.L, notspd);
    RPYW_HIP(hipGetLastError());

    auto dots = [&](const double* Vb, int nv, const double* vec, double* res, int sq) -> int {
        hipLaunchKernelGGL(dots_partial_kernel, dim3(kRedBlocks), dim3(256), 0, st, Vb, n3, nv, vec, n3, partial);
        RPYW_HIP(hipGetLastError());
        hipLaunchKernelGGL(dots_final_kernel, dim3(nv), dim3(256), 0, st, partial, kRedBlocks, res, sq);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    };
    const unsigned gv = grid_of(n3);

    // beta0 = |W|, v1 = W / beta0
    int rc = dots(W, 1, W, d_tmp, 1);
    if (rc) return rc;
    double beta0 = 0.0;
    int bad = 0;
    RPYW_HIP(hipMemcpyAsync(&beta0, d_tmp, sizeof(double), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipMemcpyAsync(&bad, notspd, sizeof(int), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipStreamSynchronize(st));
    if (bad) return RPYW_ENOTSPD;
    if (beta0 == 0.0) {
        RPYW_HIP(hipMemsetAsync(out, 0, n3 * sizeof(double), st));
        return RPYW_OK;
    }
    hipLaunchKernelGGL(scale_div_kernel, dim3(gv), dim3(256), 0, st, d_tmp, W, V, n3);
    RPYW_HIP(hipGetLastError());

    std::vector<double> alpha, beta, c, cprev;
    bool converged = false;
    double rel = INFINITY;
    int k = 0;
    double host_ab[2];
    for (; k < max_iter; ++k) {
        double* vk = V + (size_t)k * n3;
        if ((rc = pc.apply(2, vk, x, n3, st))) return rc;          // x = L^-T v_k
        if ((rc = products(pos, x, y, N, 1, a, eta, prec, ar, st))) return rc;  // y = M x
        if ((rc = pc.apply(1, y, w, n3, st))) return rc;           // w = L^-1 y
        if (k > 0) {
            hipLaunchKernelGGL(axpy_beta_kernel, dim3(gv), dim3(256), 0, st, d_beta + (k - 1), V + (size_t)(k - 1) * n3,
                               w, n3);
            RPYW_HIP(hipGetLastError());
        }
        for (int pass = 0; pass < 2; ++pass) {  // full reorthogonalisation, twice
            if ((rc = dots(V, k + 1, w, d_tmp, 0))) return rc;
            if (pass == 0)
                RPYW_HIP(hipMemcpyAsync(d_alpha + k, d_tmp + k, sizeof(double), hipMemcpyDeviceToDevice, st));
            hipLaunchKernelGGL(sub_vc_kernel, dim3(gv), dim3(256), 0, st, V, n3, k + 1, d_tmp, w, n3);
            RPYW_HIP(hipGetLastError());
        }
        if ((rc = dots(w, 1, w, d_beta + k, 1))) return rc;        // beta_k = |w|
        RPYW_HIP(hipMemcpyAsync(&host_ab[0], d_alpha + k, sizeof(double), hipMemcpyDeviceToHost, st));
        RPYW_HIP(hipMemcpyAsync(&host_ab[1], d_beta + k, sizeof(double), hipMemcpyDeviceToHost, st));
        RPYW_HIP(hipStreamSynchronize(st));
        const double ak = host_ab[0], bk = host_ab[1];
        alpha.push_back(ak);
        c.assign(k + 1, 0.0);
        if (tridiag_sqrt_coeffs(alpha.data(), beta.data(), k + 1, beta0, c.data()) != RPYW_OK) return RPYW_EHIP;
        if (k > 0) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i <= k; ++i) {
                const double dlt = c[i] - (i < k ? cprev[i] : 0.0);
                num += dlt * dlt;
                den += c[i] * c[i];
            }
            rel = std::sqrt(num / den);
            if (rel <= tol) {
                converged = true;
                break;
            }
        }
        const double prev_b = k > 0 ? beta[k - 1] : 0.0;
        if (bk <= 1e-14 * (std::fabs(ak) + prev_b)) {  // invariant subspace
            converged = true;
            break;
        }
        cprev = c;
        beta.push_back(bk);
        if (k + 1 < max_iter) {
            hipLaunchKernelGGL(scale_div_kernel, dim3(gv), dim3(256), 0, st, d_beta + k, w, V + (size_t)(k + 1) * n3,
                               n3);
            RPYW_HIP(hipGetLastError());
        }
    }
    const int used = (int)c.size();
    *iters = converged ? k + 1 : max_iter;
    *err = std::isfinite(rel) ? rel : 0.0;
    RPYW_HIP(hipMemcpyAsync(d_c, c.data(), used * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(vc_kernel, dim3(gv), dim3(256), 0, st, V, n3, used, d_c, y, n3);  // y = V c
    RPYW_HIP(hipGetLastError());
    if ((rc = pc.apply(0, y, out, n3, st))) return rc;  // out = L y
    RPYW_HIP(hipStreamSynchronize(st));                // c leaves scope
    return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
}

}  // namespace rpyw
