/*
 * FP64 CPU oracle for the wall-corrected Rotne-Prager-Yamakawa blob mobility.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes (arXiv:1709.02410):
 *   - the 3x3 blob-blob blocks M_ij that map a force on blob j to the
 *     velocity of blob i (Sec. II.A, definition of the blob-blob mobility),
 *     built from the Rotne-Prager-Yamakawa tensor (Sec. II.A) plus the
 *     no-slip-wall image correction of the Rotne-Prager-Blake tensor (named
 *     in Sec. II.A, used for all results of Sec. IV), with the blob-blob
 *     overlap form of the RPY tensor and a blob-wall regularisation that keeps
 *     M symmetric positive definite when blobs overlap the wall (Sec. IV,
 *     opening paragraph);
 *   - the dense product u = M f (Sec. II.A, direct dense products);
 *   - derivatives of M by forward-mode dual numbers through the same
 *     templated pair function: the vector-Jacobian product of u = M(r) f and
 *     the divergence of M that the thermal drift needs (Sec. III, random
 *     finite differences converge to it).
 *
 * The paper cites but does not print these formulas; the readings used here:
 *   Wall regularisation: z~ = max(z, a), B = min(z/a, 1),
 *       M_ij = B_i B_j Mhat(r~_i, r~_j).  (A congruence with a positive
 *       diagonal, so SPD is kept; exact agreement with the authors' form is
 *       parity unpinned, its stated properties are pinned by the tests.)
 *   Free part, in units of mu0 = 1/(6 pi eta a), d = |r~_i - r~_j|:
 *       d > 2a : (3a/(4d) + a^3/(2d^3)) I + (3a/(4d) - 3a^3/(2d^3)) e e^T
 *       d <= 2a: (1 - 9d/(32a)) I + (3d/(32a)) e e^T,  d = 0: I.
 *   Wall part: Blake's image system for a point force above a no-slip plane
 *       with the Faxen operators (1 + a^2/6 Lap) applied at target and
 *       source, written in q = e_z, p = t/rho, s = 1/rho^2 where
 *       R = r~_i - mirror(r~_j), rho = |R|/a, e = R/|R|, t = z~_j/a.
 *
 * Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no intrinsics).
 * All arrays are row-major FP64 [N][3].
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <omp.h>

namespace {

/* Forward-mode dual number with three derivative directions. */
struct Dual {
    double v;
    double d[3];
};

inline Dual mk(double v) { return Dual{v, {0.0, 0.0, 0.0}}; }
inline Dual operator+(const Dual& a, const Dual& b) {
    return Dual{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
inline Dual operator-(const Dual& a, const Dual& b) {
    return Dual{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
inline Dual operator-(const Dual& a) { return Dual{-a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
inline Dual operator*(const Dual& a, const Dual& b) {
    Dual r;
    r.v = a.v * b.v;
    for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
    Dual r;
    r.v = a.v / b.v;
    for (int k = 0; k < 3; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
inline Dual operator+(const Dual& a, double c) { return a + mk(c); }
inline Dual operator+(double c, const Dual& a) { return mk(c) + a; }
inline Dual operator-(const Dual& a, double c) { return a - mk(c); }
inline Dual operator-(double c, const Dual& a) { return mk(c) - a; }
inline Dual operator*(const Dual& a, double c) {
    return Dual{a.v * c, {a.d[0] * c, a.d[1] * c, a.d[2] * c}};
}
inline Dual operator*(double c, const Dual& a) { return a * c; }
inline Dual operator/(const Dual& a, double c) { return a * (1.0 / c); }
inline Dual operator/(double c, const Dual& a) { return mk(c) / a; }
inline Dual sqrt(const Dual& a) {
    double s = std::sqrt(a.v);
    Dual r;
    r.v = s;
    for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] / (2.0 * s);
    return r;
}

inline double sqrt(double x) { return std::sqrt(x); }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
template <class S> S cst(double c);
template <> double cst<double>(double c) { return c; }
template <> Dual cst<Dual>(double c) { return mk(c); }

/* Free-space RPY tensor with the overlap form, in units of mu0.
 * dv = r~_i - r~_j.  Coincident blobs (d = 0) give the identity with zero
 * derivative (the limit of the overlap branch). */
template <class S>
void rpy_free(const S dv[3], double a, S out[3][3]) {
    S d2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    if (val(d2) == 0.0) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) out[i][j] = cst<S>(i == j ? 1.0 : 0.0);
        return;
    }
    S d = sqrt(d2);
    S c1, c2;
    if (val(d) > 2.0 * a) {
        S ad = a / d;
        S ad3 = ad * ad * ad;
        c1 = 0.75 * ad + 0.5 * ad3;
        c2 = 0.75 * ad - 1.5 * ad3;
    } else {
        c1 = 1.0 - (9.0 / 32.0) * d / a;
        c2 = (3.0 / 32.0) * d / a;
    }
    S e[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[i][j] = c2 * e[i] * e[j] + (i == j ? c1 : cst<S>(0.0));
}

/* No-slip wall correction of the Rotne-Prager-Blake tensor, units of mu0.
 * rt: (regularised) target position, rs: (regularised) source position.
 * Holds for every pair including the self pair (R = 2 z ez there). */
template <class S>
void rpb_wall(const S rt[3], const S rs[3], double a, S out[3][3]) {
    S R[3] = {rt[0] - rs[0], rt[1] - rs[1], rt[2] + rs[2]};
    S Rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    S rho = Rn / a;
    S e[3] = {R[0] / Rn, R[1] / Rn, R[2] / Rn};
    S q = e[2];
    S t = rs[2] / a;
    S p = t / rho;
    S s = 1.0 / (rho * rho);
    S q2 = q * q, q3 = q2 * q, q4 = q2 * q2, p2 = p * p, s2 = s * s;
    S A = (-0.75 - 1.5 * q * p + 1.5 * p2 + 0.5 * (3.0 * q2 - 1.0) * s + 0.5 * (1.0 - 5.0 * q2) * s2) / rho;
    S B = (-0.75 + 4.5 * q * p - 4.5 * p2 + 0.5 * (3.0 - 15.0 * q2) * s + 0.5 * (35.0 * q2 - 5.0) * s2) / rho;
    S U = -0.75 * q + 1.5 * p;
    S V = -4.5 * q2 * p + 4.5 * q * p2 + 0.5 * (15.0 * q3 - 3.0 * q) * s + 0.5 * (15.0 * q - 35.0 * q3) * s2;
    S C = (U + V) / rho;   /* target in-plane velocity from a normal force */
    S Cp = (U - V) / rho;  /* target normal velocity from an in-plane force */
    S E = (-0.75 - 0.75 * q2 + 1.5 * q * p - 4.5 * q3 * p - 1.5 * p2 + 4.5 * q2 * p2 +
           0.5 * (15.0 * q4 - 6.0 * q2 - 1.0) * s + 0.5 * (-35.0 * q4 + 30.0 * q2 - 3.0) * s2) / rho;
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) out[i][j] = B * e[i] * e[j] + (i == j ? A : cst<S>(0.0));
        out[i][2] = C * e[i];
        out[2][i] = Cp * e[i];
    }
    out[2][2] = E;
}

/* Full regularised block M_ij / mu0 for target ri, source rj.
 * part: 0 = full, 1 = free RPY only, 2 = wall correction only (the last two
 * skip the B factors and use the regularised heights; for the pins). */
template <class S>
void pair_block(const S ri[3], const S rj[3], double a, int part, S out[3][3]) {
    S Bi = val(ri[2]) < a ? ri[2] / a : cst<S>(1.0);
    S Bj = val(rj[2]) < a ? rj[2] / a : cst<S>(1.0);
    S ti[3] = {ri[0], ri[1], val(ri[2]) < a ? cst<S>(a) : ri[2]};
    S tj[3] = {rj[0], rj[1], val(rj[2]) < a ? cst<S>(a) : rj[2]};
    S fr[3][3], wl[3][3];
    S dv[3] = {ti[0] - tj[0], ti[1] - tj[1], ti[2] - tj[2]};
    rpy_free(dv, a, fr);
    rpb_wall(ti, tj, a, wl);
    if (part == 1) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) out[i][j] = fr[i][j];
        return;
    }
    if (part == 2) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) out[i][j] = wl[i][j];
        return;
    }
    S bb = Bi * Bj;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[i][j] = bb * (fr[i][j] + wl[i][j]);
}

inline double mu0(double a, double eta) { return 1.0 / (6.0 * M_PI * eta * a); }

}  // namespace

extern "C" {

/* One 3x3 block, scaled by mu0 (part 0) or in mu0 units (parts 1, 2).
 * out is row-major: out[3*row + col], row = velocity, col = force. */
void oracle_pair_block(const double* ri, const double* rj, double a, double eta, int part, double* out) {
    double o[3][3];
    pair_block<double>(ri, rj, a, part, o);
    double sc = part == 0 ? mu0(a, eta) : 1.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 * i + j] = sc * o[i][j];
}

/* u = M f on selected target rows (rows == NULL: all N rows, u is [N][3];
 * otherwise u is [nrows][3] in the order of rows).  Plain double loop over
 * (target, source) pairs, OpenMP over target rows (Sec. II.A). */
void oracle_matvec(const double* pos, const double* f, double* u, int64_t N, double a, double eta,
                   const int64_t* rows, int64_t nrows, int nthreads) {
    const double m0 = mu0(a, eta);
    const int64_t nr = rows ? nrows : N;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows ? rows[r] : r;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            double blk[3][3];
            pair_block<double>(pos + 3 * i, pos + 3 * j, a, 0, blk);
            for (int c = 0; c < 3; ++c)
                acc[c] += blk[c][0] * f[3 * j] + blk[c][1] * f[3 * j + 1] + blk[c][2] * f[3 * j + 2];
        }
        for (int c = 0; c < 3; ++c) u[3 * r + c] = m0 * acc[c];
    }
}

/* Source blob j as seen from target i in the pseudo-periodic domain
 * (Sec. IV.B, dense suspensions): the minimum image of r_j, shifted by
 * (n_x + sx) Lx and (n_y + sy) Ly with n the nearest integer to
 * (r_i - r_j) / L (ties to even) and sx, sy in {-1, 0, 1}. */
static void periodic_image(const double* ri, const double* rj, double Lx, double Ly, int sx, int sy, double* out) {
    const double nx = std::nearbyint((ri[0] - rj[0]) / Lx), ny = std::nearbyint((ri[1] - rj[1]) / Ly);
    out[0] = rj[0] + (nx + sx) * Lx;
    out[1] = rj[1] + (ny + sy) * Ly;
    out[2] = rj[2];
}

/* u = M f in the pseudo-periodic domain: for every (target, source) pair
 * the source's minimum image and the 8 periodic images around it (the self
 * pair included: the blob itself and its 8 images). */
void oracle_matvec_periodic(const double* pos, const double* f, double* u, int64_t N, double a, double eta,
                            double Lx, double Ly, const int64_t* rows, int64_t nrows, int nthreads) {
    const double m0 = mu0(a, eta);
    const int64_t nr = rows ? nrows : N;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows ? rows[r] : r;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j)
            for (int sx = -1; sx <= 1; ++sx)
                for (int sy = -1; sy <= 1; ++sy) {
                    double rj[3], blk[3][3];
                    periodic_image(pos + 3 * i, pos + 3 * j, Lx, Ly, sx, sy, rj);
                    pair_block<double>(pos + 3 * i, rj, a, 0, blk);
                    for (int c = 0; c < 3; ++c)
                        acc[c] += blk[c][0] * f[3 * j] + blk[c][1] * f[3 * j + 1] + blk[c][2] * f[3 * j + 2];
                }
        for (int c = 0; c < 3; ++c) u[3 * r + c] = m0 * acc[c];
    }
}

/* Dense pseudo-periodic M (row-major 3N x 3N), for tiny N. */
void oracle_dense_periodic(const double* pos, int64_t N, double a, double eta, double Lx, double Ly,
                           double* out) {
    const double m0 = mu0(a, eta);
    const int64_t n3 = 3 * N;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double sum[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int sx = -1; sx <= 1; ++sx)
                for (int sy = -1; sy <= 1; ++sy) {
                    double rj[3], blk[3][3];
                    periodic_image(pos + 3 * i, pos + 3 * j, Lx, Ly, sx, sy, rj);
                    pair_block<double>(pos + 3 * i, rj, a, 0, blk);
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c) sum[r][c] += blk[r][c];
                }
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) out[(3 * i + r) * n3 + 3 * j + c] = m0 * sum[r][c];
        }
}

/* Dense 3N x 3N matrix M (row-major), for tiny N. */
void oracle_dense(const double* pos, int64_t N, double a, double eta, double* out) {
    const double m0 = mu0(a, eta);
    const int64_t n3 = 3 * N;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double blk[3][3];
            pair_block<double>(pos + 3 * i, pos + 3 * j, a, 0, blk);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) out[(3 * i + r) * n3 + 3 * j + c] = m0 * blk[r][c];
        }
}

/* Vector-Jacobian product of u = M(r) f for the scalar L = sum_i g_i . u_i.
 * grad_f = M g (M is symmetric).  grad_pos_k = sum_j [g_k^T d1M(r_k, r_j) f_j
 * + f_k^T d1M(r_k, r_j) g_j], with d1 the derivative in the first (target)
 * argument of the full regularised block, taken with dual numbers; the
 * j = k term yields the total derivative of the self block by reciprocity.
 * rows == NULL: every blob k, outputs [N][3]; otherwise only blobs rows[r],
 * outputs [nrows][3] in the order of rows. */
void oracle_vjp(const double* pos, const double* f, const double* g, int64_t N, double a, double eta,
                double* grad_pos, double* grad_f, const int64_t* rows, int64_t nrows, int nthreads) {
    const double m0 = mu0(a, eta);
    const int64_t nr = rows ? nrows : N;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t k = rows ? rows[r] : r;
        Dual rk[3];
        for (int c = 0; c < 3; ++c) {
            rk[c] = mk(pos[3 * k + c]);
            rk[c].d[c] = 1.0;
        }
        double gp[3] = {0.0, 0.0, 0.0};
        double gf[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            Dual rj[3] = {mk(pos[3 * j]), mk(pos[3 * j + 1]), mk(pos[3 * j + 2])};
            Dual blk[3][3];
            pair_block<Dual>(rk, rj, a, 0, blk);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    const double w = g[3 * k + r] * f[3 * j + c] + f[3 * k + r] * g[3 * j + c];
                    for (int dd = 0; dd < 3; ++dd) gp[dd] += blk[r][c].d[dd] * w;
                    gf[r] += blk[r][c].v * g[3 * j + c];
                }
        }
        for (int c = 0; c < 3; ++c) {
            grad_pos[3 * r + c] = m0 * gp[c];
            grad_f[3 * r + c] = m0 * gf[c];
        }
    }
}

/* Divergence of M: div_i,a = sum_j sum_b dM_{ij,ab} / d r_{j,b}.
 * For j != i the derivative acts on the source argument; for j = i both
 * arguments move (total derivative of the self block). */
void oracle_divergence(const double* pos, int64_t N, double a, double eta, double* div, int nthreads) {
    const double m0 = mu0(a, eta);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            Dual rj[3];
            for (int c = 0; c < 3; ++c) {
                rj[c] = mk(pos[3 * j + c]);
                rj[c].d[c] = 1.0;
            }
            Dual ri[3];
            if (j == i) {
                for (int c = 0; c < 3; ++c) ri[c] = rj[c];
            } else {
                for (int c = 0; c < 3; ++c) ri[c] = mk(pos[3 * i + c]);
            }
            Dual blk[3][3];
            pair_block<Dual>(ri, rj, a, 0, blk);
            for (int r = 0; r < 3; ++r)
                for (int b = 0; b < 3; ++b) acc[r] += blk[r][b].d[b];
        }
        for (int c = 0; c < 3; ++c) div[3 * i + c] = m0 * acc[c];
    }
}

}  /* extern "C" */
