// Driver for a sanitizer build (-fsanitize=address,undefined) of the FP64
// oracle (oracle/rpy_oracle.cpp, linked as a separate object): every entry
// point on small random inputs that include blobs below the wall,
// overlapping and coincident pairs, with cross-checks between the entry
// points (dense matrix against products, selected rows against all rows,
// symmetry).  Exits non-zero on a failed check; the sanitizers abort on any
// memory or undefined-behaviour error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
void oracle_pair_block(const double* ri, const double* rj, double a, double eta, int part, double* out);
void oracle_matvec(const double* pos, const double* f, double* u, int64_t N, double a, double eta,
                   const int64_t* rows, int64_t nrows, int nthreads);
void oracle_matvec_periodic(const double* pos, const double* f, double* u, int64_t N, double a, double eta,
                            double Lx, double Ly, const int64_t* rows, int64_t nrows, int nthreads);
void oracle_dense(const double* pos, int64_t N, double a, double eta, double* out);
void oracle_dense_periodic(const double* pos, int64_t N, double a, double eta, double Lx, double Ly, double* out);
void oracle_vjp(const double* pos, const double* f, const double* g, int64_t N, double a, double eta,
                double* grad_pos, double* grad_f, const int64_t* rows, int64_t nrows, int nthreads);
void oracle_divergence(const double* pos, int64_t N, double a, double eta, double* div, int nthreads);
}

static int fails = 0;
static void expect(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++fails;
    }
}

int main() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::normal_distribution<double> G(0.0, 1.0);
    const int N = 37;
    const double a = 0.9, eta = 1.3, Lx = 11.0, Ly = 12.5;
    std::vector<double> pos(3 * N), f(3 * N), g(3 * N);
    for (int i = 0; i < N; ++i) {
        pos[3 * i] = 10.0 * U(rng);
        pos[3 * i + 1] = 10.0 * U(rng);
        pos[3 * i + 2] = 0.2 + 3.0 * U(rng);  // some below z = a
        for (int c = 0; c < 3; ++c) {
            f[3 * i + c] = G(rng);
            g[3 * i + c] = G(rng);
        }
    }
    for (int c = 0; c < 3; ++c) pos[3 * 2 + c] = pos[3 * 1 + c];  // coincident pair
    pos[3 * 3] = pos[3 * 4] + 0.3;                                  // overlapping pair
    pos[3 * 3 + 1] = pos[3 * 4 + 1];
    pos[3 * 3 + 2] = pos[3 * 4 + 2];
    const int n3 = 3 * N;
    for (int per = 0; per < 2; ++per) {
        std::vector<double> M((size_t)n3 * n3), u(n3), ur(3 * 5);
        if (per)
            oracle_dense_periodic(pos.data(), N, a, eta, Lx, Ly, M.data());
        else
            oracle_dense(pos.data(), N, a, eta, M.data());
        double asym = 0.0, scale = 0.0;
        for (int i = 0; i < n3; ++i)
            for (int j = 0; j < n3; ++j) {
                asym = std::fmax(asym, std::fabs(M[(size_t)i * n3 + j] - M[(size_t)j * n3 + i]));
                scale = std::fmax(scale, std::fabs(M[(size_t)i * n3 + j]));
            }
        expect(asym <= 1e-14 * scale, "dense matrix symmetric");
        if (per)
            oracle_matvec_periodic(pos.data(), f.data(), u.data(), N, a, eta, Lx, Ly, nullptr, 0, 2);
        else
            oracle_matvec(pos.data(), f.data(), u.data(), N, a, eta, nullptr, 0, 2);
        double err = 0.0, us = 0.0;
        for (int i = 0; i < n3; ++i) {
            double s = 0.0;
            for (int j = 0; j < n3; ++j) s += M[(size_t)i * n3 + j] * f[j];
            err = std::fmax(err, std::fabs(s - u[i]));
            us = std::fmax(us, std::fabs(u[i]));
        }
        expect(err <= 1e-13 * us, "product equals dense matrix times force");
        const int64_t rows[5] = {36, 0, 3, 3, 17};
        if (per)
            oracle_matvec_periodic(pos.data(), f.data(), ur.data(), N, a, eta, Lx, Ly, rows, 5, 1);
        else
            oracle_matvec(pos.data(), f.data(), ur.data(), N, a, eta, rows, 5, 1);
        for (int r = 0; r < 5; ++r)
            for (int c = 0; c < 3; ++c) expect(ur[3 * r + c] == u[3 * rows[r] + c], "selected rows equal all rows");
    }
    std::vector<double> gp(n3), gf(n3), gpr(6), gfr(6), div(n3), blk(9);
    oracle_vjp(pos.data(), f.data(), g.data(), N, a, eta, gp.data(), gf.data(), nullptr, 0, 2);
    const int64_t vr[2] = {5, 30};
    oracle_vjp(pos.data(), f.data(), g.data(), N, a, eta, gpr.data(), gfr.data(), vr, 2, 1);
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            expect(gpr[3 * r + c] == gp[3 * vr[r] + c] && gfr[3 * r + c] == gf[3 * vr[r] + c], "VJP rows");
    oracle_divergence(pos.data(), N, a, eta, div.data(), 2);
    bool finite = true;
    for (int i = 0; i < n3; ++i) finite = finite && std::isfinite(gp[i]) && std::isfinite(div[i]);
    expect(finite, "finite derivatives");
    for (int part = 0; part < 3; ++part) {
        oracle_pair_block(&pos[3 * 3], &pos[3 * 4], a, eta, part, blk.data());
        for (double v : blk) expect(std::isfinite(v), "finite pair block");
    }
    std::printf(fails ? "sanitize-oracle: %d failures\n" : "sanitize-oracle: ok\n", fails);
    return fails ? 1 : 0;
}
