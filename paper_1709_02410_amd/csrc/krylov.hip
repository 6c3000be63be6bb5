// Building blocks shared by the Krylov solvers (preconditioned Lanczos for
// M^{1/2} W and GMRES for the rigid-body saddle-point system,
// arXiv:1709.02410 Sec. II): the block-diagonal preconditioner factors
// (Sec. II.B: per body, the dense block M^(pp) of that body alone, other
// bodies ignored, wall kept, and its Cholesky factor), and FP64 vector
// kernels (update, dot products with a fixed-order finish, combination).
// All reductions use a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "pair_math.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

constexpr int kBodyThreads = 128;
constexpr int kBuildThreads = 256;

// Dense M^(pp) of one body (units: physical, includes mu0 and B factors)
// assembled in LDS, then factorised in place (right-looking Cholesky).  The
// LDS is sized at launch for the largest body of the call (ld = 3 n_max + 1
// doubles per row, then 4 n_max doubles of blob data), so that small bodies
// keep many workgroups per CU.
template <int KR>
__global__ __launch_bounds__(kBuildThreads) void precond_build_kernel(const double* __restrict__ pos,
                                                                     const int* __restrict__ bofs,
                                                                     const int64_t* __restrict__ lofs, double inv_a,
                                                                     double mu0, double* __restrict__ Lout,
                                                                     int* __restrict__ notspd, int nmax) {
    extern __shared__ double lds[];
    const int ld = 3 * nmax + 1;
    double* Abase = lds;
    double* px = lds + 3 * nmax * ld;
    double* py = px + nmax;
    double* pz = py + nmax;
    double* pb = pz + nmax;
    // KR > 0: the eliminated identity Y (n x n, row stride 3 nmax), after
    // the blob data
    double* Ybase = pb + nmax;
    const int ldy = 3 * nmax;
    __shared__ int bad;
    const int p = blockIdx.x;
    const int b0 = bofs[p], nb = bofs[p + 1] - b0, n = 3 * nb;
#define A(i, j) Abase[(i) * ld + (j)]
#define Y(i, j) Ybase[(i) * ldy + (j)]
    if (threadIdx.x == 0) bad = 0;
    if constexpr (KR > 0)
        for (int q = threadIdx.x; q < n * n; q += blockDim.x) Y(q / n, q % n) = q / n == q % n ? 1.0 : 0.0;
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
            for (int al = 0; al < 3; ++al) A(3 * ia + al, 3 * ib + beta) = sc * u[al];
        }
    }
    __syncthreads();
    // One barrier per column: step k updates the trailing lower triangle
    // with the unscaled column, A(i, j) -= A(i, k) A(j, k) / A(k, k), then
    // scales column k by 1 / sqrt(A(k, k)) (one reciprocal, then products);
    // the scaling touches only column k, which no later step reads or
    // writes, so it needs no barrier of its own.
    // Threads form a 16 x 16 grid over (row, column) of the trailing block.
    // For bodies of up to 16 blobs (KR = 3 rows and columns per thread) a
    // thread loads its column-k values and its entries first, then updates
    // and stores them, so that its LDS reads overlap; the same steps also
    // eliminate an identity block Y, which yields L^-1 without a separate
    // substitution (below).
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    for (int k = 0; k < n; ++k) {
        const double d = A(k, k);
        const bool ok = d > 0.0;
        if constexpr (KR > 0) {
            // every load is issued unconditionally from an in-bounds entry
            // (row and column clamped to n - 1) and masked afterwards, so
            // that the loads go out together instead of one branch each
            const int nl = n - 1;
            double ai[KR], aj[KR], v[KR][KR];
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                const int i = k + 1 + tr + 16 * r, j = k + 1 + tc + 16 * r;
                ai[r] = A(i < n ? i : nl, k);
                aj[r] = A(j < n ? j : nl, k);
            }
#pragma unroll
            for (int r = 0; r < KR; ++r)
#pragma unroll
                for (int c = 0; c < KR; ++c) {
                    const int i = k + 1 + tr + 16 * r, j = k + 1 + tc + 16 * c;
                    v[r][c] = A(i < n ? i : nl, j < n ? j : nl);
                }
            // the same row operations on Y (rows i > k, columns j <= k, the
            // only nonzero ones): Y(i, j) -= (A(i, k) / A(k, k)) Y(k, j)
            double yk[KR], yv[KR][KR];
#pragma unroll
            for (int c = 0; c < KR; ++c) {
                const int j = tc + 16 * c;
                yk[c] = Y(k, j < n ? j : nl);
            }
#pragma unroll
            for (int r = 0; r < KR; ++r)
#pragma unroll
                for (int c = 0; c < KR; ++c) {
                    const int i = k + 1 + tr + 16 * r, j = tc + 16 * c;
                    yv[r][c] = Y(i < n ? i : nl, j < n ? j : nl);
                }
            const double id = ok ? 1.0 / d : 0.0;
#pragma unroll
            for (int r = 0; r < KR; ++r)
#pragma unroll
                for (int c = 0; c < KR; ++c) {
                    const int i = k + 1 + tr + 16 * r, j = k + 1 + tc + 16 * c, jy = tc + 16 * c;
                    if (j <= i && i < n) A(i, j) = v[r][c] - ai[r] * aj[c] * id;
                    if (jy <= k && i < n) Y(i, jy) = yv[r][c] - ai[r] * id * yk[c];
                }
        } else {
            const double id = ok ? 1.0 / d : 0.0;
            for (int i = k + 1 + tr; i < n; i += 16) {
                const double aik = A(i, k);
                for (int j = k + 1 + tc; j <= i; j += 16) A(i, j) -= aik * A(j, k) * id;
            }
        }
        __syncthreads();
        const double sd = ok ? sqrt(d) : 1.0, isd = 1.0 / sd;
        for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A(i, k) *= isd;
        if (threadIdx.x == 0) {
            if (!ok) bad = 1;
            A(k, k) = sd;
        }
    }
    __syncthreads();
    // reciprocals of the diagonal of L (the inverse's diagonal), in the free
    // position-staging area
    double* rd = px;  // 4 nmax >= n doubles
    for (int i = threadIdx.x; i < n; i += blockDim.x) rd[i] = 1.0 / A(i, i);
    __syncthreads();
    double* L = Lout + 2 * lofs[p];
    double* Li = L + (int64_t)n * n;
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int i = q / n, j = q % n;
        L[q] = j <= i ? A(i, j) : 0.0;
    }
    if constexpr (KR > 0) {
        // A = L1 D L1^T with L1 unit lower triangular; the elimination turned
        // the identity into Y = L1^-1, and L = L1 D^{1/2}, so L^-1 =
        // D^{-1/2} Y: row i of Y times 1 / L(i, i)
        for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
            const int i = q / n, j = q % n;
            Li[q] = j <= i ? Y(i, j) * rd[i] : 0.0;
        }
        if (threadIdx.x == 0 && bad) atomicOr(notspd, 1);
        return;
    }
    // Inverse factor L^-1 (lower triangular), four lanes per column: forward
    // substitution of L x = e_col, entry (i, col) = -(sum over col <= k < i
    // of L(i, k) x_k) / L(i, i), the lanes taking k = col + lane (mod 4) and
    // adding their shares in a fixed butterfly (all four get the same sum).
    // Entry (i, col), i > col, is kept in the free upper triangle of A at
    // (col, i), a row only this lane group touches (one wave), written by its
    // first lane and read by all four in later rows: LDS operations of one
    // wave complete in order, and every later read of the row follows the
    // write in program order.
    {
        const int sub = threadIdx.x & 3;
        for (int col = threadIdx.x >> 2; col < n; col += kBuildThreads / 4) {
            const double xc = rd[col];
            for (int i = col + 1; i < n; ++i) {
                double s = 0.0;
                for (int k = col + sub; k < i; k += 4) s += A(i, k) * (k == col ? xc : A(col, k));
                s += __shfl_xor(s, 1, 4);
                s += __shfl_xor(s, 2, 4);
                const double x = -s * rd[i];
                if (sub == 0) A(col, i) = x;
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int i = q / n, j = q % n;
        Li[q] = i > j ? A(j, i) : i == j ? rd[i] : 0.0;
    }
    if (threadIdx.x == 0 && bad) atomicOr(notspd, 1);
#undef A
#undef Y
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
                                                                     double* __restrict__ out,
                                                                     const double* __restrict__ V, int64_t ld,
                                                                     const double* __restrict__ c, int nc) {
    __shared__ double x[3 * kMaxBodyBlobs];
    const int p = blockIdx.x;
    const int e0 = 3 * bofs[p], n = 3 * bofs[p + 1] - e0;
    const double* F = Lall + 2 * lofs[p] + (mode == 0 ? 0 : (int64_t)n * n);
    const double inv = scale ? 1.0 / scale[0] : 1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double vr = nc > 0 ? minus_comb(v, V, ld, c, nc, e0 + i) : v[e0 + i];
        const double vi = scale ? vr * inv : vr;
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
                                  double* __restrict__ out, const double* __restrict__ V,
                                  const double* __restrict__ c, int nc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    const double vr = nc > 0 ? minus_comb(v, V, n3, c, nc, e) : v[e];
    const double vi = scale ? vr * (1.0 / scale[0]) : vr;
    if (store) store[e] = vi;
    out[e] = mode == 0 ? ldiag[e] * vi : vi / ldiag[e];
}

// Blocking of the dot products: a block of 256 threads takes 256 m
// consecutive entries (m per thread, 1 <= m <= kDotPerThread), with m as
// small as keeps the grid at kDotBlocks blocks or fewer.
constexpr int kDotBlocks = 1024;
constexpr int kDotPerThread = 8;

__host__ __device__ inline int dot_per_thread(int64_t n) {
    const int64_t m = (n + 256 * (int64_t)kDotBlocks - 1) / (256 * (int64_t)kDotBlocks);
    return (int)(m < 1 ? 1 : m > kDotPerThread ? kDotPerThread : m);
}

// Sum over groups of G consecutive lanes (G a power of two up to 64; fixed
// butterfly order); every lane of a group gets its group's sum.
template <int G>
__device__ __forceinline__ double group_sum(double s) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

constexpr int kDotBatch = 16;

// Last block of update_dots_kernel: out[j] = sum of partial[j][0..nblk) for
// j < nd (square root when nv == 0), TPV threads per vector, each adding the
// blocks b = its index (mod TPV) in order (eight loads in flight), then a
// TPV-lane butterfly.
template <int TPV>
__device__ __forceinline__ void finish_dots(const double* __restrict__ partial, int nblk, int nd, int nv,
                                            int copy_idx, double* __restrict__ out, double* cpv) {
    constexpr int kPass = 256 / TPV;
    const int jq = threadIdx.x / TPV, q = threadIdx.x % TPV;
    for (int j0 = 0; j0 < nd; j0 += kPass) {
        const int j = j0 + jq;
        double s = 0.0;
        if (j < nd) {
            const double* pj = partial + (int64_t)j * nblk;
            for (int b = q; b < nblk; b += 8 * TPV) {
                double v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = b + i * TPV < nblk ? pj[b + i * TPV] : 0.0;
#pragma unroll
                for (int i = 0; i < 8; ++i) s += v[i];
            }
        }
        s = group_sum<TPV>(s);
        if (q == 0 && j < nd) {
            const double r = nv > 0 ? s : sqrt(s);
            out[j] = r;
            if (j == copy_idx) *cpv = r;
        }
    }
}

// Update then dot products in one pass:
//   w = win - bscale[0] vprev - sum_{j < nsub} csub[j] V_j  (each term only
//   when given; written to wout unless there is nothing to write),
//   out[j] = V_j . w (j < nv), or out[0] = |w| when nv == 0.
// A block takes 256 m consecutive entries (blockIdx.x) and one group of
// kDotBatch vectors (blockIdx.y; several groups run as separate blocks,
// each repeating the update of its entries, and only group 0 writes wout,
// which therefore must not be win when there are several groups and an
// update).  Dot products go kDotBatch vectors at a time: every thread puts
// its entries' products into an LDS tile, then 16 threads per vector add 16
// tile columns each and a 16-lane butterfly finishes the block partial,
// partial[j][blockIdx.x].  The last block
// to finish (one atomic ticket, no waiting) adds each j's partials
// (finish_dots) into out[j], copies out[copy_idx] to copy_to and re-arms the
// ticket.  Every sum has a fixed order.
__global__ __launch_bounds__(256) void update_dots_kernel(const double* win, double* wout, int64_t n, int m,
                                                          const double* vprev, const double* __restrict__ bscale,
                                                          const double* V, int64_t ld,
                                                          const double* __restrict__ csub, int nsub, int nv,
                                                          double* __restrict__ partial, unsigned* __restrict__ ticket,
                                                          double* __restrict__ out, int copy_idx,
                                                          double* __restrict__ copy_to, double* hdst,
                                                          const double* hsrc, int nh, int with_norm,
                                                          double* beta_out) {
    __shared__ double tile[kDotBatch][257];
    __shared__ double cpv;
    __shared__ bool last;
    const int t = threadIdx.x;
    const int nblk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * 256 * m + t;
    const bool upd = vprev || nsub > 0;
    double x[kDotPerThread];
#pragma unroll
    for (int r = 0; r < kDotPerThread; ++r) {
        const int64_t e = base + (int64_t)r * 256;
        x[r] = 0.0;
        if (r >= m || e >= n) continue;
        double v = win[e];
        if (vprev) v -= bscale[0] * vprev[e];
        int j = 0;
        // sixteen loads in flight before their terms are subtracted (in
        // order): the long reorthogonalisation updates are latency-bound
        for (; j + 15 < nsub; j += 16) {
            double av[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) av[u] = V[(j + u) * ld + e];
#pragma unroll
            for (int u = 0; u < 16; ++u) v -= csub[j + u] * av[u];
        }
        for (; j + 3 < nsub; j += 4) {
            const double a0 = V[j * ld + e], a1 = V[(j + 1) * ld + e];
            const double a2 = V[(j + 2) * ld + e], a3 = V[(j + 3) * ld + e];
            v -= csub[j] * a0;
            v -= csub[j + 1] * a1;
            v -= csub[j + 2] * a2;
            v -= csub[j + 3] * a3;
        }
        for (; j < nsub; ++j) v -= csub[j] * V[j * ld + e];
        if (wout && (upd || wout != win) && blockIdx.y == 0) wout[e] = v;
        x[r] = v;
    }
    const int nd = nv > 0 ? nv + (with_norm ? 1 : 0) : 1;  // results: dots, then |w|^2 or |w|
    const int jr = t >> 4, c0 = t & 15;  // reduction: vector jr of the batch, columns c0 + 16 i
    const int jend = (int)(blockIdx.y + 1) * kDotBatch < nd ? (int)(blockIdx.y + 1) * kDotBatch : nd;
    for (int j0 = (int)blockIdx.y * kDotBatch; j0 < jend; j0 += kDotBatch) {
        const int jn = nd - j0 < kDotBatch ? nd - j0 : kDotBatch;
#pragma unroll
        for (int u = 0; u < kDotBatch; ++u) {
            double p = 0.0;
            if (u < jn) {
                if (j0 + u < nv) {
                    const double* a = V + (j0 + u) * ld;
#pragma unroll
                    for (int r = 0; r < kDotPerThread; ++r) {
                        const int64_t e = base + (int64_t)r * 256;
                        if (r < m && e < n) p = fma(a[e], x[r], p);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < kDotPerThread; ++r) p = fma(x[r], x[r], p);
                }
            }
            tile[u][t] = p;
        }
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) s += tile[jr][c0 + 16 * i];
        s = group_sum<16>(s);
        if (c0 == 0 && jr < jn) partial[(int64_t)(j0 + jr) * nblk + blockIdx.x] = s;
        __syncthreads();
    }
    __threadfence();
    if (t == 0) last = atomicAdd(ticket, 1u) == (unsigned)(nblk * gridDim.y) - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (nd <= 4)
        finish_dots<64>(partial, nblk, nd, nv, copy_idx, out, &cpv);
    else if (nd <= 16)
        finish_dots<16>(partial, nblk, nd, nv, copy_idx, out, &cpv);
    else
        finish_dots<4>(partial, nblk, nd, nv, copy_idx, out, &cpv);
    __syncthreads();
    if (t == 0) {
        double cp = cpv;
        if (beta_out) {
            double s2 = out[nv];
            for (int j = 0; j < nv; ++j) s2 -= out[j] * out[j];
            cp = s2 > 0.0 ? sqrt(s2) : 0.0;
            *beta_out = cp;
        }
        if (copy_to) copy_to[0] = cp;
        *ticket = 0u;
    }
    if (nh > 0) {
        __syncthreads();
        for (int i = t; i < nh; i += 256) hdst[i] = hsrc[i];
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

}  // namespace

int64_t dot_chunks(int64_t n) {
    const int64_t span = 256 * (int64_t)dot_per_thread(n);
    return (n + span - 1) / span;
}

int vec_update_dots(const double* win, double* wout, int64_t n, const double* vprev, const double* bscale,
                    const double* V, int64_t ld, const double* csub, int nsub, int nv, double* partial,
                    unsigned* ticket, double* out, int copy_idx, double* copy_to, hipStream_t st, double* hdst,
                    const double* hsrc, int nh, bool with_norm, double* beta_out) {
    if (nh < 0 || (nh > 0 && (!hdst || !hsrc))) return RPYW_EINVAL;
    if ((with_norm || beta_out) && nv < 1) return RPYW_EINVAL;
    if (beta_out && !with_norm) return RPYW_EINVAL;
    // vector groups as separate blocks (more of the GPU for few entries and
    // many vectors), unless an in-place update forbids it
    const bool upd = vprev || nsub > 0;
    const int nd = nv > 0 ? nv + (with_norm ? 1 : 0) : 1;
    const int ngrp = (upd && win == wout) ? 1 : (nd + kDotBatch - 1) / kDotBatch;
    hipLaunchKernelGGL(update_dots_kernel, dim3((unsigned)dot_chunks(n), (unsigned)ngrp), dim3(256), 0, st, win,
                       wout, n, dot_per_thread(n), vprev, bscale, V, ld, csub, nsub, nv, partial, ticket, out,
                       copy_idx, copy_to, hdst, hsrc, nh, with_norm ? 1 : 0, beta_out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int vec_dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* partial, unsigned* ticket,
             double* out, int copy_idx, double* copy_to, hipStream_t st) {
    return vec_update_dots(w, nullptr, n, nullptr, nullptr, V, ld, nullptr, 0, nv, partial, ticket, out, copy_idx,
                           copy_to, st);
}

int vec_comb(const double* V, int64_t ld, int nv, const double* c, double* out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(vc_kernel, dim3(grid_of(n)), dim3(256), 0, st, V, ld, nv, c, out, n);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int BodyFactors::apply(int mode, const double* v, double* out, int64_t n3, hipStream_t st, const double* scale,
                       double* store, const double* V, const double* c, int nc) const {
    if (nc < 0 || (nc > 0 && (!V || !c))) return RPYW_EINVAL;
    if (diag)
        hipLaunchKernelGGL(diag_apply_kernel, dim3(grid_of(n3)), dim3(256), 0, st, L, n3, mode, v, scale, store, out,
                           V, c, nc);
    else
        hipLaunchKernelGGL(precond_apply_kernel, dim3(nb), dim3(kBodyThreads), 0, st, L, bofs, lofs, mode, v, scale,
                           store, out, V, n3, c, nc);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

size_t body_factors_bytes(int64_t N, int n_bodies) {
    if (n_bodies == 0) return align_up((size_t)3 * N * sizeof(double));
    // sum over bodies of 2 (3 n_p)^2 <= 18 N max_p n_p
    const size_t lsz = (size_t)18 * std::min<int64_t>(N, kMaxBodyBlobs) * N;
    return align_up((size_t)(n_bodies + 1) * sizeof(int)) + align_up((size_t)(n_bodies + 1) * sizeof(int64_t)) +
           align_up(lsz * sizeof(double));
}

void body_factors_tables(const int64_t* body_offsets, int n_bodies, std::vector<int>& hb, std::vector<int64_t>& hl,
                         int* nmax) {
    hb.assign(n_bodies + 1, 0);
    hl.assign(n_bodies + 1, 0);
    *nmax = 1;
    for (int p = 0; p <= n_bodies; ++p) hb[p] = (int)body_offsets[p];
    for (int p = 0; p < n_bodies; ++p) {
        const int64_t nbl = body_offsets[p + 1] - body_offsets[p];
        hl[p + 1] = hl[p] + 9 * nbl * nbl;
        *nmax = std::max(*nmax, (int)nbl);
    }
}

int body_factors_launch(const double* pos, int64_t N, double a, double eta, const BodyFactors& pc, int nmax,
                        int* notspd, hipStream_t st) {
    const double inv_a = 1.0 / a, m0 = 1.0 / (6.0 * M_PI * eta * a);
    if (!pc.diag) {
        const size_t lds = ((size_t)3 * nmax * (3 * nmax + 1) + 4 * (size_t)nmax) * sizeof(double);
        if (3 * nmax <= 48) {
            const size_t ldsy = lds + (size_t)9 * nmax * nmax * sizeof(double);  // and Y
            hipLaunchKernelGGL(precond_build_kernel<3>, dim3(pc.nb), dim3(kBuildThreads), ldsy, st, pos, pc.bofs,
                               pc.lofs, inv_a, m0, pc.L, notspd, nmax);
        } else {
            if (lds > 65536)  // up to 129 KB for 42-blob bodies
                RPYW_HIP(hipFuncSetAttribute((const void*)precond_build_kernel<0>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(precond_build_kernel<0>, dim3(pc.nb), dim3(kBuildThreads), lds, st, pos, pc.bofs,
                               pc.lofs, inv_a, m0, pc.L, notspd, nmax);
        }
    } else {
        hipLaunchKernelGGL(blob_diag_kernel, dim3(grid_of(N)), dim3(256), 0, st, pos, N, inv_a, m0, pc.L, notspd);
    }
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int body_factors_build(const double* pos, int64_t N, double a, double eta, const int64_t* body_offsets, int n_bodies,
                       Arena& ar, hipStream_t st, BodyFactors& pc, int* notspd) {
    pc.diag = n_bodies == 0;
    pc.nb = n_bodies;
    pc.flag = notspd;
    int nmax = 1;
    if (!pc.diag) {
        std::vector<int> hb;
        std::vector<int64_t> hl;
        body_factors_tables(body_offsets, n_bodies, hb, hl, &nmax);
        // both tables in one upload: lofs, then bofs
        const size_t lb = align_up(hl.size() * sizeof(int64_t));
        std::vector<char> tab(lb + hb.size() * sizeof(int));
        std::memcpy(tab.data(), hl.data(), hl.size() * sizeof(int64_t));
        std::memcpy(tab.data() + lb, hb.data(), hb.size() * sizeof(int));
        char* dtab = (char*)ar.take(tab.size());
        pc.L = (double*)ar.take((size_t)2 * hl[n_bodies] * sizeof(double));  // L and L^-1
        if (!dtab || !pc.L) return RPYW_ENOMEM;
        pc.lofs = (int64_t*)dtab;
        pc.bofs = (int*)(dtab + lb);
        if (int r = stage_upload(tab.data(), tab.size(), dtab, st)) return r;
    } else {
        pc.L = (double*)ar.take((size_t)3 * N * sizeof(double));
        if (!pc.L) return RPYW_ENOMEM;
    }
    return body_factors_launch(pos, N, a, eta, pc, nmax, notspd, st);
}

// ---------------------------------------------------------- staging ring

namespace {

// Pinned ring buffer for small host -> device uploads: an upload takes the
// next free stretch, copied from host memory the caller may free at once;
// a stretch is reused only after the copy that last read it has completed
// (its event), so uploads normally never wait.
struct StageRing {
    std::mutex mu;
    char* host = nullptr;
    size_t cap = 0, head = 0;
    struct Use {
        size_t off, len;
        hipEvent_t ev;
    };
    std::vector<Use> busy;
    std::vector<hipEvent_t> idle;
};
StageRing g_ring;

}  // namespace

int stage_upload(const void* src, size_t bytes, void* dst, hipStream_t st) {
    if (bytes == 0) return RPYW_OK;
    std::lock_guard<std::mutex> lk(g_ring.mu);
    const size_t len = align_up(bytes);
    auto retire = [&](size_t lo, size_t hi) -> int {  // wait for uses overlapping [lo, hi)
        for (size_t i = 0; i < g_ring.busy.size();) {
            const StageRing::Use u = g_ring.busy[i];
            if (u.off < hi && lo < u.off + u.len) {
                RPYW_HIP(hipEventSynchronize(u.ev));
                g_ring.idle.push_back(u.ev);
                g_ring.busy.erase(g_ring.busy.begin() + (long)i);
            } else {
                ++i;
            }
        }
        return RPYW_OK;
    };
    // completed copies (oldest first) free their stretch without waiting
    while (!g_ring.busy.empty() && hipEventQuery(g_ring.busy.front().ev) == hipSuccess) {
        g_ring.idle.push_back(g_ring.busy.front().ev);
        g_ring.busy.erase(g_ring.busy.begin());
    }
    if (len > g_ring.cap) {
        if (int r = retire(0, g_ring.cap)) return r;
        if (g_ring.host) RPYW_HIP(hipHostFree(g_ring.host));
        g_ring.host = nullptr;
        g_ring.cap = g_ring.head = 0;
        const size_t cap = std::max(len * 4, (size_t)1 << 20);
        RPYW_HIP(hipHostMalloc((void**)&g_ring.host, cap, hipHostMallocDefault));
        g_ring.cap = cap;
    }
    if (g_ring.head + len > g_ring.cap) g_ring.head = 0;
    const size_t off = g_ring.head;
    if (int r = retire(off, off + len)) return r;
    hipEvent_t ev;
    if (!g_ring.idle.empty()) {
        ev = g_ring.idle.back();
        g_ring.idle.pop_back();
    } else {
        RPYW_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    std::memcpy(g_ring.host + off, src, bytes);
    RPYW_HIP(hipMemcpyAsync(dst, g_ring.host + off, bytes, hipMemcpyHostToDevice, st));
    RPYW_HIP(hipEventRecord(ev, st));
    g_ring.busy.push_back({off, len, ev});
    g_ring.head = off + len;
    return RPYW_OK;
}

int PinnedSlots::reserve(size_t bytes) {
    cur ^= 1;
    Bank& k = bank[cur];
    if (k.tail) RPYW_HIP(hipEventSynchronize(k.tail));
    if (k.cap < bytes) {
        if (k.p) RPYW_HIP(hipHostFree(k.p));
        k.p = nullptr;
        k.cap = 0;
        k.dp = nullptr;
        // fine-grained (coherent) so that kernel stores reach host memory
        // without passing through the GPU caches
        RPYW_HIP(hipHostMalloc((void**)&k.p, bytes, hipHostMallocMapped | hipHostMallocCoherent));
        RPYW_HIP(hipHostGetDevicePointer((void**)&k.dp, k.p, 0));
        k.cap = bytes;
    }
    for (auto& e : k.ev)
        if (!e) RPYW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    p = k.p;
    dp = k.dp;
    ev = k.ev;
    return RPYW_OK;
}

int PinnedSlots::release(hipStream_t st) {
    Bank& k = bank[cur];
    if (!k.tail) RPYW_HIP(hipEventCreateWithFlags(&k.tail, hipEventDisableTiming));
    RPYW_HIP(hipEventRecord(k.tail, st));
    return RPYW_OK;
}

}  // namespace rpyw
