// Preconditioned Lanczos for Brownian blob displacements M^{1/2} W
// (arXiv:1709.02410, Sec. II.B).
//
//   L     block diagonal, one lower Cholesky factor per body of the dense
//         block M^(pp) of that body alone (other bodies ignored, wall kept);
//         built once per call (Sec. II.B, block-diagonal preconditioner).
//   G     = L^-1 M L^-T, applied as L^-T -> product by M -> L^-1.
//   Krylov basis V (FP64, [iter][3N]), three-term recurrence with full
//   reorthogonalisation (two classical Gram-Schmidt passes), alpha/beta kept
//   on the device; one device->host copy of (alpha_k, beta_k) per iteration
//   into pinned memory.  Iteration k + 1 only needs beta_k on the device, so
//   it is queued before the host has examined iteration k and is discarded
//   if k turns out to be the last: the host solve overlaps the GPU work.
//   Host: eigendecomposition of the k x k tridiagonal T_k, coefficients
//   c_k = beta0 Q Lambda^{1/2} Q^T e1; since V is orthonormal the stopping
//   test |y_k - y_{k-1}| <= tol |y_k| is evaluated on c.  At the end
//   out = L (V c).
// All reductions are two-stage with a fixed order (bitwise reproducible).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "pair_math.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

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
    double* L = Lout + 2 * lofs[p];
    double* Li = L + (int64_t)n * n;
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int i = q / n, j = q % n;
        L[q] = j <= i ? A[i][j] : 0.0;
    }
    // Inverse factor L^-1 (lower triangular), one column per thread: forward
    // substitution of L x = e_col, the column written to global memory.
    for (int col = threadIdx.x; col < n; col += blockDim.x) {
        for (int i = 0; i < col; ++i) Li[i * n + col] = 0.0;
        double xc = 1.0 / A[col][col];
        Li[col * n + col] = xc;
        for (int i = col + 1; i < n; ++i) {
            double s = 0.0;
            for (int k = col; k < i; ++k) s += A[i][k] * Li[k * n + col];
            Li[i * n + col] = -s / A[i][i];
        }
    }
    if (threadIdx.x == 0 && bad) atomicOr(notspd, 1);
}

// mode 0: out = L v;  1: out = L^-1 v;  2: out = L^-T v, with the factor L
// and its inverse Li stored per body (both lower triangular, n x n).  One
// workgroup per body, one output entry per thread (dense triangular
// mat-vec).  With `scale`, the input is v / scale[0] and, with `store`, that
// scaled input is also written there (this forms the next Lanczos vector
// v_{k+1} = w / beta_k).
__global__ __launch_bounds__(kBodyThreads) void precond_apply_kernel(const double* __restrict__ Lall,
                                                                     const int* __restrict__ bofs,
                                                                     const int64_t* __restrict__ lofs, int mode,
                                                                     const double* __restrict__ v,
                                                                     const double* __restrict__ scale,
                                                                     double* __restrict__ store,
                                                                     double* __restrict__ out) {
    __shared__ double x[3 * kMaxBodyBlobs];
    const int p = blockIdx.x;
    const int e0 = 3 * bofs[p], n = 3 * bofs[p + 1] - e0;
    const double* F = Lall + 2 * lofs[p] + (mode == 0 ? 0 : (int64_t)n * n);
    const double inv = scale ? 1.0 / scale[0] : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double vi = scale ? v[e0 + i] * inv : v[e0 + i];
        x[i] = vi;
        if (store) store[e0 + i] = vi;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        if (mode == 2)
            for (int j = i; j < n; ++j) s += F[j * n + i] * x[j];  // (L^-1)^T row i
        else
            for (int j = 0; j <= i; ++j) s += F[i * n + j] * x[j];
        out[e0 + i] = s;
    }
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

// mode 0: out = D v; 1, 2: out = v / D (diagonal L); scale/store as above.
__global__ void diag_apply_kernel(const double* __restrict__ ldiag, int64_t n3, int mode, const double* __restrict__ v,
                                  const double* __restrict__ scale, double* __restrict__ store,
                                  double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    const double vi = scale ? v[e] * (1.0 / scale[0]) : v[e];
    if (store) store[e] = vi;
    out[e] = mode == 0 ? ldiag[e] * vi : vi / ldiag[e];
}

// w_out = w_in - bscale[0] * vprev - sum_{j < nsub} csub[j] V_j (each term
// only when given).
__global__ void update_kernel(const double* __restrict__ win, double* __restrict__ wout, int64_t n3,
                              const double* __restrict__ vprev, const double* __restrict__ bscale,
                              const double* __restrict__ V, int64_t ld, const double* __restrict__ csub, int nsub) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    double x = win[e];
    if (vprev) x -= bscale[0] * vprev[e];
    for (int j = 0; j < nsub; ++j) x -= csub[j] * V[j * ld + e];
    wout[e] = x;
}

constexpr int kDotChunk = 2048;  // entries per dot-product block (8 per thread)

// Dot products V_j . w (j < nv), or w . w when nv == 0, on a 2-D grid of
// (chunk, j) blocks; block partials go to partial[j][chunk].  The last block
// to finish (one atomic ticket, no waiting) adds each j's partials in chunk
// order (one thread per j) into out[j] (square root for the norm), copies
// out[copy_idx] to copy_to, and re-arms the ticket.
__global__ __launch_bounds__(256) void dots_kernel(const double* __restrict__ V, int64_t ld, int nv,
                                                   const double* __restrict__ w, int64_t n3,
                                                   double* __restrict__ partial, unsigned* __restrict__ ticket,
                                                   double* __restrict__ out, int copy_idx,
                                                   double* __restrict__ copy_to) {
    __shared__ double red[256];
    __shared__ bool last;
    const int j = blockIdx.y, nchunk = gridDim.x;
    const double* a = nv > 0 ? V + j * ld : w;
    const int64_t e0 = (int64_t)blockIdx.x * kDotChunk + threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kDotChunk / 256; ++r) {
        const int64_t e = e0 + r * 256;
        if (e < n3) s += a[e] * w[e];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)j * nchunk + blockIdx.x] = red[0];
    __threadfence();
    if (threadIdx.x == 0) last = atomicAdd(ticket, 1u) == gridDim.x * gridDim.y - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int nd = gridDim.y;
    for (int jj = threadIdx.x; jj < nd; jj += blockDim.x) {
        const double* p = partial + (int64_t)jj * nchunk;
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        int c = 0;
        for (; c + 3 < nchunk; c += 4) {
            t0 += p[c];
            t1 += p[c + 1];
            t2 += p[c + 2];
            t3 += p[c + 3];
        }
        for (; c < nchunk; ++c) t0 += p[c];
        const double t = (t0 + t1) + (t2 + t3);
        out[jj] = nv > 0 ? t : sqrt(t);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (copy_to) copy_to[0] = out[copy_idx];
        *ticket = 0u;
    }
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

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }
int64_t dot_chunks(int64_t n3) { return (n3 + kDotChunk - 1) / kDotChunk; }

// Pinned host slots for the per-iteration (alpha_k, beta_k) copies, so the
// copies are truly asynchronous; one Lanczos call uses them at a time.
struct PinnedAB {
    std::mutex mu;
    double* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
PinnedAB g_ab;

struct Precond {
    bool diag = true;
    int nb = 0;
    int* bofs = nullptr;
    int64_t* lofs = nullptr;
    double* L = nullptr;  // factors (bodies) or diagonal [3N]

    int apply(int mode, const double* v, double* out, int64_t n3, hipStream_t st, const double* scale = nullptr,
              double* store = nullptr) const {
        if (diag)
            hipLaunchKernelGGL(diag_apply_kernel, dim3(grid_of(n3)), dim3(256), 0, st, L, n3, mode, v, scale, store,
                               out);
        else
            hipLaunchKernelGGL(precond_apply_kernel, dim3(nb), dim3(kBodyThreads), 0, st, L, bofs, lofs, mode, v,
                               scale, store, out);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    }
};

}  // namespace

// ---------------------------------------------------- tridiagonal (host)

// Implicit symmetric QL with Wilkinson shifts on T = tridiag(e, d, e)
// (Golub & Van Loan, Sec. 8.3).  The eigenvector matrix is the product
// Z = G_1 G_2 ... G_M of the plane rotations the sweeps apply; only
// Z^T e1 (its first row) and products Z v are needed, so the rotations are
// recorded and the first row is tracked instead of accumulating Z: O(k^2)
// work per solve instead of O(k^3).  Returns false if an eigenvalue needs
// more than 60 sweeps.
struct Rot {
    int i;
    double c, s;
};

// sqrt(a^2 + b^2); the entries of T are O(1) (eigenvalues of the
// preconditioned mobility), far from overflow, so no rescaling is needed.
static inline double pyth(double a, double b) { return std::sqrt(a * a + b * b); }

static bool tridiag_ql(std::vector<double>& d, std::vector<double>& e, std::vector<double>& row0,
                       std::vector<Rot>& rots, int k) {
    row0.assign(k, 0.0);
    row0[0] = 1.0;
    rots.clear();
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
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = pyth(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = pyth(f, g);
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
                // Z <- Z G with G = [[c, s], [-s, c]] on columns (i, i+1)
                rots.push_back({i, c, s});
                const double zi = row0[i], zi1 = row0[i + 1];
                row0[i + 1] = s * zi + c * zi1;
                row0[i] = c * zi - s * zi1;
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
    std::vector<double> d(alpha, alpha + k), e(k, 0.0), row0;
    std::vector<Rot> rots;
    for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
    if (!tridiag_ql(d, e, row0, rots, k)) return RPYW_NOT_CONVERGED;
    // c = beta0 Z (Lambda^{1/2} Z^T e1) = beta0 G_1 (G_2 (... (G_M v)))
    for (int i = 0; i < k; ++i) c[i] = beta0 * std::sqrt(std::max(d[i], 0.0)) * row0[i];
    for (size_t t = rots.size(); t-- > 0;) {
        const Rot& g = rots[t];
        const double vi = c[g.i], vi1 = c[g.i + 1];
        c[g.i] = g.c * vi + g.s * vi1;
        c[g.i + 1] = -g.s * vi + g.c * vi1;
    }
    return RPYW_OK;
}

// ---------------------------------------------------- driver

size_t lanczos_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec) {
    const size_t n3 = (size_t)3 * N;
    size_t b = 0;
    b += align_up((size_t)(n_bodies + 1) * sizeof(int));
    b += align_up((size_t)(n_bodies + 1) * sizeof(int64_t));
    const size_t lsz = n_bodies > 0 ? (size_t)18 * std::min<int64_t>(N, kMaxBodyBlobs) * N : n3;
    b += align_up(lsz * sizeof(double));
    b += align_up((size_t)(max_iter + 1) * n3 * sizeof(double));  // V
    b += 3 * align_up(n3 * sizeof(double));                        // x, y, w
    b += align_up((size_t)(max_iter + 2) * dot_chunks(n3) * sizeof(double));
    b += 4 * align_up((size_t)2 * (max_iter + 8) * sizeof(double));  // alpha/beta, c1, c2, b0
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
        pc.L = (double*)ar.take((size_t)2 * hl[n_bodies] * sizeof(double));  // L and L^-1
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
    const int64_t nchunk = dot_chunks(n3);
    double* partial = (double*)ar.take((size_t)(max_iter + 2) * nchunk * sizeof(double));
    double* d_ab = (double*)ar.take(2 * (max_iter + 8) * sizeof(double));  // alpha_k, beta_k interleaved
    double* d_c1 = (double*)ar.take(2 * (max_iter + 8) * sizeof(double));
    double* d_c2 = (double*)ar.take(2 * (max_iter + 8) * sizeof(double));
    double* d_b0 = (double*)ar.take(8 * sizeof(double));
    unsigned* ticket = (unsigned*)ar.take(kAlign);
    notspd = (int*)ar.take(sizeof(int));
    if (!V || !x || !y || !w || !partial || !d_ab || !d_c1 || !d_c2 || !d_b0 || !ticket || !notspd)
        return RPYW_ENOMEM;
    std::lock_guard<std::mutex> lk(g_ab.mu);
    const size_t need = (size_t)2 * (max_iter + 2) * sizeof(double);
    if (g_ab.cap < need) {
        if (g_ab.p) RPYW_HIP(hipHostFree(g_ab.p));
        g_ab.p = nullptr;
        g_ab.cap = 0;
        RPYW_HIP(hipHostMalloc((void**)&g_ab.p, need, hipHostMallocDefault));
        g_ab.cap = need;
    }
    for (auto& e : g_ab.ev)
        if (!e) RPYW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    double* h_ab = g_ab.p;

    RPYW_HIP(hipMemsetAsync(notspd, 0, sizeof(int), st));
    RPYW_HIP(hipMemsetAsync(ticket, 0, sizeof(unsigned), st));
    if (pc.diag)
        hipLaunchKernelGGL(blob_diag_kernel, dim3(grid_of(N)), dim3(256), 0, st, pos, N, inv_a, m0, pc.L, notspd);
    else
        hipLaunchKernelGGL(precond_build_kernel, dim3(n_bodies), dim3(kBodyThreads), 0, st, pos, pc.bofs, pc.lofs,
                           inv_a, m0, pc.L, notspd);
    RPYW_HIP(hipGetLastError());

    const unsigned gv = grid_of(n3);
    auto update = [&](const double* vprev, const double* bscale, const double* csub, int nsub) -> int {
        hipLaunchKernelGGL(update_kernel, dim3(gv), dim3(256), 0, st, w, w, n3, vprev, bscale, V, n3, csub, nsub);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    };
    // dot products with V_0..V_{nv-1} (nv > 0) or the norm (nv = 0) of vec
    auto dots = [&](const double* vec, int nv, double* res, int copy_idx, double* copy_to) -> int {
        hipLaunchKernelGGL(dots_kernel, dim3((unsigned)nchunk, (unsigned)(nv > 0 ? nv : 1)), dim3(256), 0, st, V, n3,
                           nv, vec, n3, partial, ticket, res, copy_idx, copy_to);
        RPYW_HIP(hipGetLastError());
        return RPYW_OK;
    };

    // beta0 = |W|
    int rc = dots(W, 0, d_b0, 0, nullptr);
    if (rc) return rc;
    double beta0 = 0.0;
    int bad = 0;
    RPYW_HIP(hipMemcpyAsync(&beta0, d_b0, sizeof(double), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipMemcpyAsync(&bad, notspd, sizeof(int), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipStreamSynchronize(st));
    if (bad) return RPYW_ENOTSPD;
    if (beta0 == 0.0) {
        RPYW_HIP(hipMemsetAsync(out, 0, n3 * sizeof(double), st));
        return RPYW_OK;
    }

    // Enqueue iteration k on the GPU: it needs beta_{k-1} only on the device,
    // so iteration k + 1 is queued before the host has decided whether
    // iteration k converged (its results are discarded if so).
    auto launch_iter = [&](int k) -> int {
        double* vk = V + (size_t)k * n3;
        int r;
        if (k == 0)
            r = pc.apply(2, W, x, n3, st, d_b0, vk);  // v_0 = W / beta0, x = L^-T v_0
        else
            r = pc.apply(2, w, x, n3, st, d_ab + 2 * (k - 1) + 1, vk);  // v_k = w / beta_{k-1}
        if (r) return r;
        if ((r = products(pos, x, y, N, 1, a, eta, prec, ar, st))) return r;  // y = M x
        if ((r = pc.apply(1, y, w, n3, st))) return r;                        // w = L^-1 y
        // w -= beta_{k-1} v_{k-1}; full reorthogonalisation in two passes,
        // alpha_k = v_k . w from the first
        if (k > 0 && (r = update(V + (size_t)(k - 1) * n3, d_ab + 2 * (k - 1) + 1, nullptr, 0))) return r;
        if ((r = dots(w, k + 1, d_c1, k, d_ab + 2 * k))) return r;
        if ((r = update(nullptr, nullptr, d_c1, k + 1))) return r;
        if ((r = dots(w, k + 1, d_c2, 0, nullptr))) return r;
        if ((r = update(nullptr, nullptr, d_c2, k + 1))) return r;
        if ((r = dots(w, 0, d_ab + 2 * k + 1, 0, nullptr))) return r;  // beta_k = |w|
        RPYW_HIP(hipMemcpyAsync(h_ab + 2 * k, d_ab + 2 * k, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        RPYW_HIP(hipEventRecord(g_ab.ev[k & 1], st));
        return RPYW_OK;
    };

    std::vector<double> alpha, beta, c, cprev;
    bool converged = false;
    double rel = INFINITY;
    int k = 0;
    if ((rc = launch_iter(0))) return rc;
    for (; k < max_iter; ++k) {
        RPYW_HIP(hipEventSynchronize(g_ab.ev[k & 1]));
        const double ak = h_ab[2 * k], bk = h_ab[2 * k + 1];
        if (k + 1 < max_iter && (rc = launch_iter(k + 1))) return rc;
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
    }
    const int used = (int)c.size();
    *iters = converged ? k + 1 : max_iter;
    *err = std::isfinite(rel) ? rel : 0.0;
    RPYW_HIP(hipMemcpyAsync(d_c1, c.data(), used * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(vc_kernel, dim3(gv), dim3(256), 0, st, V, n3, used, d_c1, y, n3);  // y = V c
    RPYW_HIP(hipGetLastError());
    if ((rc = pc.apply(0, y, out, n3, st))) return rc;  // out = L y
    RPYW_HIP(hipStreamSynchronize(st));                // c leaves scope
    return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
}

}  // namespace rpyw
