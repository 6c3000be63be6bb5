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
//   for small problems it is queued before the host has examined iteration
//   k and is discarded if k turns out to be the last: the host solve
//   overlaps the GPU work.
//   Host: the coefficients c_k = beta0 T_k^{1/2} e1 of the k x k
//   tridiagonal T_k (= beta0 Q Lambda^{1/2} Q^T e1 for T_k = Q Lambda Q^T);
//   since V is orthonormal the stopping test |y_k - y_{k-1}| <= tol |y_k| is
//   evaluated on c.  At the end out = L (V c).
// All reductions are two-stage with a fixed order (bitwise reproducible).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "rpyw_internal.h"

namespace rpyw {

namespace {

// Pinned host slots for the per-iteration (alpha_k, beta_k) copies; one
// Lanczos call uses them at a time.
PinnedSlots g_ab;

}  // namespace

// ---------------------------------------------------- tridiagonal (host)

// Eigen-decomposition T = Z Lambda Z^T of the symmetric tridiagonal
// T = tridiag(e, d, e) (d: diagonal, e[i] = T(i, i+1)) by the implicit
// symmetric QR algorithm with Wilkinson shifts (Golub & Van Loan, Sec. 8.3:
// the implicit shifted QR step, Alg. 8.3.2, inside the deflating driver of
// Alg. 8.3.3).  Each step chases a bulge down the trailing unreduced block
// with plane rotations T <- Q^T T Q, Q = [[c, -s], [s, c]] on rows and
// columns (i, i+1); Z is the product of all the Q's.  Only Z^T e1 (the first
// row of Z) and one product Z v are needed, so the rotations are recorded
// and the first row is updated as they are made, instead of accumulating Z:
// O(k^2) work per solve instead of O(k^3).  Returns false if the driver
// needs more than 30 k steps.
struct Rot {
    int i;
    double c, s;
};

// sqrt(a^2 + b^2); the entries of T are O(1) (eigenvalues of the
// preconditioned mobility), far from overflow, so no rescaling is needed.
static inline double pyth(double a, double b) { return std::sqrt(a * a + b * b); }

// Whether e[i] is negligible next to its two diagonal neighbours.
static inline bool negligible(const std::vector<double>& d, const std::vector<double>& e, int i) {
    return std::fabs(e[i]) <= 1e-16 * (std::fabs(d[i]) + std::fabs(d[i + 1]));
}

static bool tridiag_eig(std::vector<double>& d, std::vector<double>& e, std::vector<double>& row0,
                        std::vector<Rot>& rots, int k) {
    row0.assign(k, 0.0);
    row0[0] = 1.0;
    rots.clear();
    e.resize(k);
    int steps = 0;
    int hi = k - 1;  // last row of the trailing block that is not yet diagonal
    while (hi > 0) {
        if (negligible(d, e, hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;  // first row of the unreduced block that ends at hi
        while (lo > 0 && !negligible(d, e, lo - 1)) --lo;
        if (++steps > 30 * k) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closer
        // to its last diagonal entry.
        const double half = 0.5 * (d[hi - 1] - d[hi]);
        const double b2 = e[hi - 1] * e[hi - 1];
        const double mu = d[hi] - b2 / (half + (half >= 0.0 ? 1.0 : -1.0) * pyth(half, e[hi - 1]));
        // Implicit QR step: the first rotation acts on (d[lo] - mu, e[lo]);
        // every later one removes the bulge T(i - 1, i + 1) it left behind.
        double x = d[lo] - mu, z = e[lo];
        for (int i = lo; i < hi; ++i) {
            const double r = pyth(x, z);
            const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? z / r : 0.0;
            if (i > lo) e[i - 1] = r;
            const double a = d[i], b = e[i], dd = d[i + 1];
            d[i] = c * c * a + 2.0 * c * s * b + s * s * dd;
            d[i + 1] = s * s * a - 2.0 * c * s * b + c * c * dd;
            e[i] = (c * c - s * s) * b + c * s * (dd - a);
            if (i + 1 < hi) {
                z = s * e[i + 1];  // new bulge T(i, i + 2)
                e[i + 1] *= c;
                x = e[i];
            }
            rots.push_back({i, c, s});
            const double zi = row0[i], zi1 = row0[i + 1];
            row0[i] = c * zi + s * zi1;
            row0[i + 1] = c * zi1 - s * zi;
        }
    }
    return true;
}

// Whether T - shift I is positive definite: its LDL^T factorisation
// (Sturm sequence) has positive pivots only.
static bool shifted_pd(const double* a, const double* b, int k, double shift) {
    double p = a[0] - shift;
    if (!(p > 0.0)) return false;
    for (int i = 1; i < k; ++i) {
        p = a[i] - shift - b[i - 1] * b[i - 1] / p;
        if (!(p > 0.0)) return false;
    }
    return true;
}

// x = T^-1 v for the SPD tridiagonal T (elimination without pivoting, which
// is stable for SPD T); wk holds 2k doubles.
static void tridiag_solve(const double* a, const double* b, int k, const double* v, double* x, double* wk) {
    double* mul = wk;
    double* piv = wk + k;
    piv[0] = a[0];
    x[0] = v[0];
    for (int i = 1; i < k; ++i) {
        mul[i - 1] = b[i - 1] / piv[i - 1];
        piv[i] = a[i] - b[i - 1] * mul[i - 1];
        x[i] = v[i] - mul[i - 1] * x[i - 1];
    }
    x[k - 1] /= piv[k - 1];
    for (int i = k - 2; i >= 0; --i) x[i] = x[i] / piv[i] - mul[i] * x[i + 1];
}

// x = T v.
static void tridiag_mul(const double* a, const double* b, int k, const double* v, double* x) {
    for (int i = 0; i < k; ++i)
        x[i] = (i > 0 ? b[i - 1] * v[i - 1] : 0.0) + a[i] * v[i] + (i + 1 < k ? b[i] * v[i + 1] : 0.0);
}

// c = beta0 T^{1/2} e1 for an SPD tridiagonal T by quadrature instead of an
// eigendecomposition (whose rotation sweeps are one long dependent chain,
// O(k^2) rotations: 0.1-0.2 ms at k = 60 on the host, longer than a GPU
// step).  T^{1/2} e1 = T T^{-1/2} e1, with
//   T^{-1/2} = (2/pi) int_0^inf (s^2 I + T)^{-1} ds
//            = (2/pi) int_R e^u (e^{2u} I + T)^{-1} du        (s = e^u).
// For one eigenvalue l the integrand is l^{-1/2} sech(u - log(l)/2) / 2:
// analytic in the strip |Im u| < pi/2 and decaying like e^{-|u|}, so the
// trapezoidal rule of step h has relative error about 2 pi exp(-pi^2 / h)
// for every eigenvalue alike (the exponentially convergent trapezoidal
// rule: Trefethen & Weideman, SIAM Review 56, 2014).  h = 1/4
// gives ~1e-17.  The nodes span the spectrum's bounds (lo <= lambda_min
// from a Sturm test, hi >= lambda_max by Gershgorin) widened by 5.5 on
// each side; the rest of the node sum, where e^{2u} is far below lo or far
// above hi, is the geometric sum of the first three terms of the series
// (s^2 I + T)^{-1} = sum_m (-s^2)^m T^{-m-1} = sum_m (-1)^m T^m s^{-2m-2}
// (neglected terms below (e^{-11})^3 of the tail).  Every node is one
// shifted tridiagonal solve; the nodes are independent, so they run in
// blocks with the node as the inner loop.  Returns false when T is not
// positive definite or too ill-conditioned for this.
static bool tridiag_sqrt_quadrature(const double* a, const double* b, int k, double beta0, double* c) {
    constexpr int NB = 16;  // nodes per block
    double hi = 0.0, amin = INFINITY;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        hi = std::max(hi, a[i] + r);
        amin = std::min(amin, a[i]);
    }
    if (!(amin > 0.0) || !std::isfinite(hi)) return false;
    double lo = 0.5 * amin;  // min_i a_i >= lambda_min
    for (int t = 0; !shifted_pd(a, b, k, lo); ++t) {
        if (t == 60) return false;
        lo *= 0.125;
    }
    // rounding in the solves near lambda_min grows with the condition
    // number: beyond hi / lo = 1e8 (errors then reach 1e-13 of the largest
    // coefficient) the eigendecomposition is used instead
    if (hi > 1e8 * lo) return false;
    const double h = 0.25, widen = 5.5, wc = (2.0 / M_PI) * h;
    const double u0 = 0.5 * std::log(lo) - widen;
    const int nn = (int)std::ceil((0.5 * std::log(hi) + widen - u0) / h) + 1;  // nodes u0 + n h, n < nn
    std::vector<double> buf((size_t)3 * k * NB + (size_t)9 * k, 0.0);
    double* mul = buf.data();                // [row][node] elimination multipliers
    double* zp = mul + (size_t)k * NB;       // [row][node] forward-eliminated right-hand side / pivot
    double* acc = zp + (size_t)k * NB;       // [row][node] weighted sums, added over nodes at the end
    double* y = acc + (size_t)k * NB;        // T^{-1/2} e1
    double* t1 = y + k;
    double* t2 = t1 + k;
    double* t3 = t2 + k;
    double* e1 = t3 + k;
    double* te = e1 + k;
    double* tte = te + k;
    double* wk = tte + k;                    // 2k
    for (int n0 = 0; n0 < nn; n0 += NB) {
        double s2[NB], w[NB], p[NB], z[NB], x[NB];
        for (int j = 0; j < NB; ++j) {
            const double u = u0 + (n0 + j) * h;
            s2[j] = std::exp(2.0 * u);
            w[j] = n0 + j < nn ? wc * std::exp(u) : 0.0;
            p[j] = s2[j] + a[0];
            z[j] = 1.0;
        }
        for (int i = 0; i + 1 < k; ++i) {
            const double bi = b[i], ai1 = a[i + 1];
            for (int j = 0; j < NB; ++j) {
                const double r = 1.0 / p[j];
                const double m = bi * r;
                zp[i * NB + j] = z[j] * r;
                mul[i * NB + j] = m;
                z[j] = -m * z[j];
                p[j] = s2[j] + ai1 - bi * m;
            }
        }
        for (int j = 0; j < NB; ++j) {
            x[j] = z[j] / p[j];
            acc[(k - 1) * NB + j] += w[j] * x[j];
        }
        for (int i = k - 2; i >= 0; --i)
            for (int j = 0; j < NB; ++j) {
                x[j] = zp[i * NB + j] - mul[i * NB + j] * x[j];
                acc[i * NB + j] += w[j] * x[j];
            }
    }
    for (int i = 0; i < k; ++i) {
        double s = 0.0;
        for (int j = 0; j < NB; ++j) s += acc[i * NB + j];
        y[i] = s;
    }
    // the node sum beyond both ends: sum over u = u0 - h, u0 - 2h, ... of
    // e^{(2m+1)u}, and over u = u0 + nn h, ... of e^{-(2m+1)u}
    e1[0] = 1.0;
    tridiag_solve(a, b, k, e1, t1, wk);
    tridiag_solve(a, b, k, t1, t2, wk);
    tridiag_solve(a, b, k, t2, t3, wk);
    tridiag_mul(a, b, k, e1, te);
    tridiag_mul(a, b, k, te, tte);
    const double uL = u0 - h, uR = u0 + nn * h;
    double gl[3], gr[3];
    for (int m = 0; m < 3; ++m) {
        const double q = 2.0 * m + 1.0, sg = (m & 1) ? -1.0 : 1.0;
        gl[m] = sg * wc * std::exp(q * uL) / (1.0 - std::exp(-q * h));
        gr[m] = sg * wc * std::exp(-q * uR) / (1.0 - std::exp(-q * h));
    }
    for (int i = 0; i < k; ++i)
        y[i] += (gl[0] * t1[i] + gl[1] * t2[i] + gl[2] * t3[i]) + (gr[0] * e1[i] + gr[1] * te[i] + gr[2] * tte[i]);
    tridiag_mul(a, b, k, y, c);
    for (int i = 0; i < k; ++i) c[i] *= beta0;
    return true;
}

// c = beta0 T^{1/2} e1: by quadrature for positive definite T of moderate
// condition, else (rounding made T indefinite, or it is very ill
// conditioned) through the eigendecomposition with the negative eigenvalues
// clamped to zero.
int tridiag_sqrt_coeffs(const double* alpha, const double* beta, int k, double beta0, double* c) {
    if (tridiag_sqrt_quadrature(alpha, beta, k, beta0, c)) return RPYW_OK;
    std::vector<double> d(alpha, alpha + k), e(k, 0.0), row0;
    std::vector<Rot> rots;
    for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
    if (!tridiag_eig(d, e, row0, rots, k)) return RPYW_NOT_CONVERGED;
    // c = beta0 Z (Lambda^{1/2} Z^T e1) = beta0 Q_1 (Q_2 (... (Q_M v)))
    for (int i = 0; i < k; ++i) c[i] = beta0 * std::sqrt(std::max(d[i], 0.0)) * row0[i];
    for (size_t t = rots.size(); t-- > 0;) {
        const Rot& g = rots[t];
        const double vi = c[g.i], vi1 = c[g.i + 1];
        c[g.i] = g.c * vi - g.s * vi1;
        c[g.i + 1] = g.s * vi + g.c * vi1;
    }
    return RPYW_OK;
}

// ---------------------------------------------------- driver

size_t lanczos_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec) {
    const size_t n3 = (size_t)3 * N;
    size_t b = body_factors_bytes(N, n_bodies);
    b += align_up((size_t)(max_iter + 1) * n3 * sizeof(double));  // V
    b += 3 * align_up(n3 * sizeof(double));                        // x, y, w
    b += align_up((size_t)(max_iter + 2) * dot_chunks(n3) * sizeof(double));
    b += 4 * align_up((size_t)2 * (max_iter + 8) * sizeof(double));  // alpha/beta, c1, c2, b0
    b += align_up(sizeof(unsigned)) + align_up(sizeof(int));        // ticket, notspd
    b += product_ws_bytes(N, prec, 1);
    // fused steps: the block partials of both Gram-Schmidt passes and the
    // workgroup tables (one unit per body or per kLanczosOutEntries / 3 blobs)
    const size_t units = (size_t)std::max<int64_t>(n_bodies, N / (kLanczosOutEntries / 3) + 1) + 1;
    int m;
    b += align_up((size_t)(max_iter + 2) * units * sizeof(double));
    b += align_up((size_t)(max_iter + 3) * lanczos_gs2_blocks((int64_t)n3, &m) * sizeof(double));
    b += align_up((units + 1) * sizeof(int)) + align_up((units + 1) * sizeof(LanczosGroup));
    b += align_up(((size_t)N / 256 + 3) * sizeof(double));  // partials of |W|^2 (padded blobs / 256)
    b += align_up(n3 * sizeof(double));                       // the summed product (large problems)
    return b + 24 * kAlign;
}

namespace {

// The Lanczos iteration with fused steps (lanczos_step.hip); same results
// as the unfused driver below up to rounding (different summation orders).
int lanczos_fused(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                  const int64_t* body_offsets, int n_bodies, double tol, int max_iter, int prec, Arena& ar, int* iters,
                  double* err, hipStream_t st, const Domain& dom, const BodyFactors* pre, const SymPlan& sp,
                  int ipw) {
    const int64_t n3 = 3 * N;
    *iters = 0;
    *err = 0.0;
    std::vector<int> h_units, h_groups;
    lanczos_units(N, body_offsets, n_bodies, h_units, h_groups);
    const int nunits = (int)h_units.size() - 1, ngroups = (int)h_groups.size() - 1;
    int m4;
    const int64_t nblk4 = lanczos_gs2_blocks(n3, &m4);
    BodyFactors pc;
    const int rw = rec_width(prec, 1);
    const int64_t npad = (int64_t)sp.ng * sp.G;
    double* V = (double*)ar.take((size_t)(max_iter + 1) * n3 * sizeof(double));
    double* y = (double*)ar.take(n3 * sizeof(double));
    double* w = (double*)ar.take(n3 * sizeof(double));
    const int64_t npack = lz_pack_blocks(npad);
    double* sqp = (double*)ar.take((size_t)npack * sizeof(double));  // partials of |W|^2
    double* part1 = (double*)ar.take((size_t)(max_iter + 2) * ngroups * sizeof(double));
    double* part2 = (double*)ar.take((size_t)(max_iter + 3) * nblk4 * sizeof(double));
    double* d_ab = (double*)ar.take(2 * (max_iter + 8) * sizeof(double));
    double* d_c = (double*)ar.take(2 * (max_iter + 8) * sizeof(double));
    int* notspd = (int*)ar.take(sizeof(int));
    // The call's small tables in one block, which the first kernel copies
    // from pinned memory: the factor tables (when the factors are built
    // here), the gather groups (units, blobs, first factor block, factor
    // size), the unit offsets.
    TableBlock tb;
    int nmax = 1;
    size_t o_lofs = 0, o_bofs = 0;
    std::vector<int64_t> hl;
    if (pre) {
        pc = *pre;
    } else {
        pc.diag = n_bodies == 0;
        pc.nb = n_bodies;
        pc.flag = notspd;
        if (!pc.diag) {
            std::vector<int> hb;
            body_factors_tables(body_offsets, n_bodies, hb, hl, &nmax);
            o_lofs = tb.add(hl.data(), hl.size() * sizeof(int64_t));
            o_bofs = tb.add(hb.data(), hb.size() * sizeof(int));
        }
    }
    size_t o_groups, o_units;
    {
        std::vector<LanczosGroup> gt(ngroups);
        int64_t loff = 0;
        for (int g = 0; g < ngroups; ++g) {
            LanczosGroup& G = gt[g];
            G.g0 = h_groups[g];
            G.g1 = h_groups[g + 1];
            G.b0 = h_units[G.g0];
            G.b1 = h_units[G.g1];
            G.loff = loff;
            G.sq = 0;
            G.pad = 0;
            if (G.g1 - G.g0 > kLanczosGroupUnits) return RPYW_EINVAL;  // not produced by lanczos_units
            for (int q = G.g0; q < G.g1; ++q) {
                const int nq = 3 * (h_units[q + 1] - h_units[q]);
                G.sq += nq * nq;
            }
            loff += G.sq;
        }
        o_groups = tb.add(gt.data(), gt.size() * sizeof(LanczosGroup));
        o_units = tb.add(h_units.data(), h_units.size() * sizeof(int));
    }
    const size_t tbytes = align_up(tb.host.size());
    tb.host.resize(tbytes, 0);
    char* d_tab = (char*)ar.take(tbytes);
    const LanczosGroup* d_groups = (const LanczosGroup*)(d_tab + o_groups);
    const int* d_units = (const int*)(d_tab + o_units);
    if (!pre) {
        pc.L = (double*)ar.take((pc.diag ? (size_t)3 * N : (size_t)2 * hl[n_bodies]) * sizeof(double));
        pc.lofs = (int64_t*)(d_tab + o_lofs);
        pc.bofs = (int*)(d_tab + o_bofs);
    }
    void* rec = ar.take((size_t)npad * rw * real_size(prec));
    double* B = (double*)ar.take((size_t)npad * sizeof(double));
    double* tpart = (double*)ar.take(sp.tpart_bytes);
    void* spart = ar.take(sp.spart_bytes);
    double* ypre = krylov_presum(sp) ? (double*)ar.take((size_t)n3 * sizeof(double)) : nullptr;
    if (!V || !y || !w || !sqp || !part1 || !part2 || !d_ab || !d_c || !notspd || !d_tab || !pc.L || !rec || !B ||
        !tpart || !spart || (krylov_presum(sp) && !ypre))
        return RPYW_ENOMEM;
    std::lock_guard<std::mutex> lk(g_ab.mu);
    const size_t hdr_bytes = align_up((size_t)(3 * (max_iter + 2) + 2) * sizeof(double));
    int rc = g_ab.reserve(hdr_bytes + tbytes);
    if (rc) return rc;
    double* h_ab = g_ab.p;
    double* dh_ab = g_ab.dp;  // the same pinned memory as kernels address it
    SlotRelease slots_done{g_ab, st};
    // the header (beta_0, then the two definiteness flags), written by vin
    // of step 0 and read by the host with step 0
    double* h_b0 = h_ab + 2 * (max_iter + 2);
    int* h_bad = (int*)(h_b0 + 1);
    double* dh_hdr = dh_ab + (h_b0 - h_ab);
    // step flags: set by the step's last kernel after alpha_k and beta_{k-1}
    // (no event per step: an event between the steps' kernels delays the next)
    double* h_flag = h_b0 + 2;
    double* dh_flag = dh_ab + (h_flag - h_ab);
    std::memset(h_flag, 0, (size_t)(max_iter + 2) * sizeof(double));
    // the tables after them
    std::memcpy((char*)h_ab + hdr_bytes, tb.host.data(), tbytes);
    const int* dh_tab = (const int*)((const char*)dh_ab + hdr_bytes);

    // positions, B, the partials of |W|^2 and the tables; clears notspd
    // before the factor build (the force slots are rewritten by every step)
    if ((rc = lz_launch_pack(prec, pos, W, N, npad, rw, a, dom, rec, B, sqp, notspd, dh_tab, (int*)d_tab,
                             (int)(tbytes / sizeof(int)), st)))
        return rc;
    if (!pre && (rc = body_factors_launch(pos, N, a, eta, pc, nmax, notspd, st))) return rc;
    const double m0 = 1.0 / (6.0 * M_PI * eta * a);

    // Step k: the product (its records written by vin of step k), w = L^-1
    // M x - beta_{k-1} v_{k-1} with the first projection, y' = w - V c1
    // with the second projection, then vin of step k + 1: beta_k, v_{k+1}
    // and the next records; it publishes step k (alpha_k, beta_k, flag).
    auto vin = [&](int k) {
        return lz_launch_vin(prec, pc, d_units, nunits, n3, k, k == 0 ? W : y, k == 0 ? sqp : part2,
                             k == 0 ? (int)npack : (int)nblk4, V, d_ab, dh_ab, dh_flag, rec, rw, B, dh_hdr, notspd,
                             pre ? pre->flag : nullptr, st);
    };
    auto launch_step = [&](int k) -> int {
        int r;
        hipEvent_t ev = nullptr;
        profile_begin(st, &ev);
        if ((r = sym_launch(rec, sp, ipw, 1, prec, a, dom, tpart, spart, st))) return r;
        profile_end(st, ev, (dom.periodic() ? 9.0 : 1.0) * (double)N * (double)N);
        if (ypre && (r = sym_finish(tpart, spart, B, N, 1, 1, prec, sp, m0, ypre, st, nullptr, 1.0 / a))) return r;
        if ((r = lz_launch_out(prec, pc, d_units, d_groups, ngroups, tpart, spart, sp, B, m0, n3, k, V, d_ab, w,
                               part1, ypre, st)))
            return r;
        if ((r = lz_launch_gs2(w, y, n3, V, k, part1, ngroups, part2, d_ab, nullptr, st))) return r;
        if ((r = vin(k + 1))) return r;  // V has room for max_iter + 1 vectors
        return RPYW_OK;
    };
    const int depth = (double)N * (double)N <= kSpeculatePairs ? kSpeculateDepth : 0;
    int queued = 0;
    auto fill = [&](int upto) -> int {  // queue steps up to index upto - 1
        for (; queued < upto && queued < max_iter; ++queued)
            if (int r = launch_step(queued)) return r;
        return RPYW_OK;
    };

    std::vector<double> alpha, beta, c, cprev;
    bool converged = false;
    double rel = INFINITY, rel1 = INFINITY, rel2 = INFINITY;
    int k = 0, used = 0;
    // host time spent waiting for steps, and steps the device had queued
    // behind the awaited one when the wait began (RPYW_LOG)
    using Clock = std::chrono::steady_clock;
    const bool logging = log_enabled();
    double wait_ms = 0.0;
    int starved = 0;
    const auto t_call = Clock::now();
    if ((rc = vin(0))) return rc;
    if ((rc = fill(1 + depth))) return rc;
    // Waits for step k: its flag in host memory, polled; the stream is
    // queried now and then so that a stream that drains without setting it
    // (a failed launch) ends the wait with an error instead of spinning.
    auto wait_step = [&](int k) -> int {
        const volatile double* f = h_flag + k;
        for (unsigned spin = 1;; ++spin) {
            if (*f != 0.0) break;
            if ((spin & 4095) == 0) {
                const hipError_t q = hipStreamQuery(st);
                if (q == hipSuccess) {
                    if (*f != 0.0) break;
                    return RPYW_EHIP;
                }
                if (q != hipErrorNotReady) return RPYW_EHIP;
            }
            __builtin_ia32_pause();
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        return RPYW_OK;
    };
    for (; k < max_iter; ++k) {
        if (logging) {
            if (queued <= k + 1) ++starved;
            const auto t0 = Clock::now();
            if ((rc = wait_step(k))) return rc;
            wait_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        } else if ((rc = wait_step(k))) {
            return rc;
        }
        if (k == 0) {
            const bool bad = h_bad[0] || h_bad[1];
            if (bad || *h_b0 == 0.0) {
                RPYW_HIP(hipStreamSynchronize(st));
                if (bad) return RPYW_ENOTSPD;
                RPYW_HIP(hipMemsetAsync(out, 0, n3 * sizeof(double), st));
                return RPYW_OK;
            }
        }
        const double ak = h_ab[2 * k], bk = h_ab[2 * k + 1];
        if (depth && (rc = fill(speculate_to(k, depth, rel1, rel2, tol) + 1))) return rc;
        alpha.push_back(ak);
        c.assign(k + 1, 0.0);
        if (tridiag_sqrt_coeffs(alpha.data(), beta.data(), k + 1, *h_b0, c.data()) != RPYW_OK) return RPYW_EHIP;
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
                used = k + 1;
                break;
            }
        }
        // beta_k ~ 0: the Krylov space is invariant (a breakdown), and this
        // step's iterate is the last
        if (bk <= 1e-14 * (std::fabs(ak) + (k > 0 ? beta[k - 1] : 0.0))) {
            converged = true;
            used = k + 1;
            break;
        }
        beta.push_back(bk);
        cprev = c;
        rel2 = rel1;
        rel1 = rel;
        if ((rc = fill(k + 2))) return rc;
    }
    if (!converged) used = max_iter;
    *iters = used;
    *err = std::isfinite(rel) ? rel : 0.0;
    if (used <= kLanczosCoefArgs) {
        // out = L (V c) in one launch, c passed by value
        if ((rc = lz_launch_fin(pc, d_units, nunits, n3, V, c.data(), used, out, st))) return rc;
    } else {
        if ((rc = stage_upload(c.data(), used * sizeof(double), d_c, st))) return rc;
        if ((rc = vec_comb(V, n3, used, d_c, y, n3, st))) return rc;  // y = V c
        if ((rc = pc.apply(0, y, out, n3, st))) return rc;            // out = L y
    }
    if (logging)
        log_line("lanczos fused steps: %d run, %d queued; host %.3f ms, of which %.3f ms waiting; %d waits with no "
                 "later step queued",
                 used, queued, std::chrono::duration<double, std::milli>(Clock::now() - t_call).count(), wait_ms,
                 starved);
    return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
}

}  // namespace

int lanczos_sqrt(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                 const int64_t* body_offsets, int n_bodies, double tol, int max_iter, int prec, Arena& ar, int* iters,
                 double* err, hipStream_t st, const Domain& dom, const BodyFactors* pre) {
    {
        SymPlan sp;
        int ipw;
        if (lanczos_fused_applies(N, prec, max_iter, dom, &sp, &ipw))
            return lanczos_fused(pos, W, out, N, a, eta, body_offsets, n_bodies, tol, max_iter, prec, ar, iters, err,
                                 st, dom, pre, sp, ipw);
    }
    const int64_t n3 = 3 * N;
    *iters = 0;
    *err = 0.0;
    BodyFactors pc;
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
    int* notspd = (int*)ar.take(sizeof(int));
    if (!V || !x || !y || !w || !partial || !d_ab || !d_c1 || !d_c2 || !d_b0 || !ticket || !notspd)
        return RPYW_ENOMEM;
    std::lock_guard<std::mutex> lk(g_ab.mu);
    int rc = g_ab.reserve((size_t)(2 * (max_iter + 2) + 2) * sizeof(double));
    if (rc) return rc;
    double* h_ab = g_ab.p;
    SlotRelease slots_done{g_ab, st};
    // beta0 and the not-positive-definite flags come back with step 0
    double* h_b0 = h_ab + 2 * (max_iter + 2);
    int* h_bad = (int*)(h_b0 + 1);

    RPYW_HIP(hipMemsetAsync(notspd, 0, sizeof(int), st));
    RPYW_HIP(hipMemsetAsync(ticket, 0, sizeof(unsigned), st));
    if (pre)
        pc = *pre;
    else if ((rc = body_factors_build(pos, N, a, eta, body_offsets, n_bodies, ar, st, pc, notspd)))
        return rc;

    // to = from - bscale[0] vprev - V csub (terms when given), then the dot
    // products of the result with V_0..V_{nv-1} (nv > 0) or its norm (nv = 0)
    auto update_dots = [&](const double* from, double* to, const double* vprev, const double* bscale,
                           const double* csub, int nsub, int nv, double* res, int copy_idx, double* copy_to) {
        return vec_update_dots(from, to, n3, vprev, bscale, V, n3, csub, nsub, nv, partial, ticket, res, copy_idx,
                               copy_to, st);
    };
    auto dots = [&](const double* vec, int nv, double* res, int copy_idx, double* copy_to) {
        return vec_dots(V, n3, nv, vec, n3, partial, ticket, res, copy_idx, copy_to, st);
    };

    // beta0 = |W|
    if ((rc = dots(W, 0, d_b0, 0, nullptr))) return rc;
    h_bad[0] = h_bad[1] = 0;
    RPYW_HIP(hipMemcpyAsync(h_b0, d_b0, sizeof(double), hipMemcpyDeviceToHost, st));
    RPYW_HIP(hipMemcpyAsync(h_bad, notspd, sizeof(int), hipMemcpyDeviceToHost, st));
    if (pre && pre->flag) RPYW_HIP(hipMemcpyAsync(h_bad + 1, pre->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    double beta0 = 0.0;

    // Enqueue iteration k on the GPU: it needs beta_{k-1} only on the device,
    // so iteration k + 1 is queued before the host has decided whether
    // iteration k converged (its results are discarded if so).
    auto launch_iter = [&](int k) -> int {
        double* vk = V + (size_t)k * n3;
        int r;
        if (k == 0)
            r = pc.apply(2, W, x, n3, st, d_b0, vk);  // v_0 = W / beta0, x = L^-T v_0
        else  // v_k = (w - V c2) / beta_{k-1}: the second correction of step k - 1
            r = pc.apply(2, w, x, n3, st, d_ab + 2 * (k - 1) + 1, vk, V, d_c2, k);
        if (r) return r;
        if ((r = products(pos, x, y, N, 1, a, eta, prec, ar, st, dom))) return r;  // y = M x
        if ((r = pc.apply(1, y, w, n3, st))) return r;                        // w = L^-1 y
        // w -= beta_{k-1} v_{k-1}; full reorthogonalisation in two passes,
        // alpha_k = v_k . w from the first (w -> y).  The second (y -> w)
        // computes c2 = V^T w and |w|^2, and beta_k = |w - V c2| from
        // |w|^2 - |c2|^2 (V orthonormal); w - V c2 itself is formed by the
        // next step's preconditioner application.  The pass also stores
        // alpha_k, beta_k into the pinned slot.
        const double* vprev = k > 0 ? V + (size_t)(k - 1) * n3 : nullptr;
        const double* bprev = k > 0 ? d_ab + 2 * (k - 1) + 1 : nullptr;
        if ((r = update_dots(w, y, vprev, bprev, nullptr, 0, k + 1, d_c1, k, d_ab + 2 * k))) return r;
        if ((r = vec_update_dots(y, w, n3, nullptr, nullptr, V, n3, d_c1, k + 1, k + 1, partial, ticket, d_c2, 0,
                                 nullptr, st, g_ab.dp + 2 * k, d_ab + 2 * k, 2, true, d_ab + 2 * k + 1)))
            return r;
        RPYW_HIP(hipEventRecord(g_ab.ev[k % PinnedSlots::kSlots], st));
        return RPYW_OK;
    };
    const int depth = (double)N * (double)N <= kSpeculatePairs ? kSpeculateDepth : 0;
    int queued = 0;
    auto fill = [&](int upto) -> int {  // queue steps up to index upto - 1
        for (; queued < upto && queued < max_iter; ++queued)
            if (int r = launch_iter(queued)) return r;
        return RPYW_OK;
    };

    std::vector<double> alpha, beta, c, cprev;
    bool converged = false;
    double rel = INFINITY, rel1 = INFINITY, rel2 = INFINITY;  // of steps k - 1, k - 2
    int k = 0;
    if ((rc = fill(1 + depth))) return rc;
    for (; k < max_iter; ++k) {
        RPYW_HIP(hipEventSynchronize(g_ab.ev[k % PinnedSlots::kSlots]));
        if (k == 0) {  // the first wait also brings beta0 and the flags
            beta0 = *h_b0;
            const bool bad = h_bad[0] || h_bad[1];
            if (bad || beta0 == 0.0) {
                RPYW_HIP(hipStreamSynchronize(st));  // drain the queued steps
                if (bad) return RPYW_ENOTSPD;
                RPYW_HIP(hipMemsetAsync(out, 0, n3 * sizeof(double), st));
                return RPYW_OK;
            }
        }
        const double ak = h_ab[2 * k], bk = h_ab[2 * k + 1];
        if (depth && (rc = fill(speculate_to(k, depth, rel1, rel2, tol) + 1))) return rc;
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
        rel2 = rel1;
        rel1 = rel;
        if ((rc = fill(k + 2))) return rc;  // step k + 1, unless queued already
    }
    const int used = (int)c.size();
    *iters = converged ? k + 1 : max_iter;
    *err = std::isfinite(rel) ? rel : 0.0;
    if ((rc = stage_upload(c.data(), used * sizeof(double), d_c1, st))) return rc;
    if ((rc = vec_comb(V, n3, used, d_c1, y, n3, st))) return rc;  // y = V c
    if ((rc = pc.apply(0, y, out, n3, st))) return rc;  // out = L y
    return converged ? RPYW_OK : RPYW_NOT_CONVERGED;
}

}  // namespace rpyw
