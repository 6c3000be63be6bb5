// CPU build of the device pair arithmetic, exported for the host tests.
#include "../../paper_1709_02410_amd/csrc/pair_math.h"

using namespace rpyw;

template <typename R>
static void block(const double* d, const double* z, double* out) {
    // out[3*row + col] = (Mhat e_col)_row, units of mu0
    PairCoef<R> c = pair_coef<R>((R)d[0], (R)d[1], (R)d[2], (R)z[0], (R)z[1]);
    for (int col = 0; col < 3; ++col) {
        R u[3] = {0, 0, 0};
        pair_apply<R>(c, (R)d[0], (R)d[1], (R)d[2], R(col == 0), R(col == 1), R(col == 2), u[0], u[1], u[2]);
        for (int r = 0; r < 3; ++r) out[3 * r + col] = (double)u[r];
    }
}

// The same block through the written-out form the matrix-core kernel
// contracts (pair_block, block_apply).
template <typename R>
static void block2(const double* d, const double* z, double* out) {
    PairCoef<R> c = pair_coef<R>((R)d[0], (R)d[1], (R)d[2], (R)z[0], (R)z[1]);
    const PairBlock<R> m = pair_block<R>(c, (R)d[0], (R)d[1], (R)d[2]);
    for (int col = 0; col < 3; ++col) {
        R u[3] = {0, 0, 0};
        block_apply<R>(m, R(col == 0), R(col == 1), R(col == 2), u[0], u[1], u[2]);
        for (int r = 0; r < 3; ++r) out[3 * r + col] = (double)u[r];
    }
}

template <typename R>
static void grad(const double* d, const double* z, const double* v12, double* out) {
    R a[3], b[3], a2[3], b2[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = (R)v12[k];
        b[k] = (R)v12[3 + k];
        a2[k] = (R)v12[6 + k];
        b2[k] = (R)v12[9 + k];
    }
    PairCoef<R> c;
    PairGrad<R> g = pair_grad<R>((R)d[0], (R)d[1], (R)d[2], (R)z[0], (R)z[1], a, b, a2, b2, &c);
    out[0] = g.dx;
    out[1] = g.dy;
    out[2] = g.dz;
    out[3] = g.rz;
    out[4] = g.zz;
    double blk[9];
    // value of a^T M b + a2^T M b2 from the returned coefficients
    double val = 0;
    for (int col = 0; col < 3; ++col) {
        R u[3] = {0, 0, 0};
        pair_apply<R>(c, (R)d[0], (R)d[1], (R)d[2], R(col == 0), R(col == 1), R(col == 2), u[0], u[1], u[2]);
        for (int r = 0; r < 3; ++r) blk[3 * r + col] = (double)u[r];
    }
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) val += v12[r] * blk[3 * r + col] * v12[3 + col] + v12[6 + r] * blk[3 * r + col] * v12[9 + col];
    out[5] = val;
}

extern "C" {
void host_block_f64(const double* d, const double* z, double* out) { block<double>(d, z, out); }
void host_block_f32(const double* d, const double* z, double* out) { block<float>(d, z, out); }
void host_block2_f64(const double* d, const double* z, double* out) { block2<double>(d, z, out); }
void host_block2_f32(const double* d, const double* z, double* out) { block2<float>(d, z, out); }
void host_grad_f64(const double* d, const double* z, const double* v, double* out) { grad<double>(d, z, v, out); }
void host_grad_f32(const double* d, const double* z, const double* v, double* out) { grad<float>(d, z, v, out); }
}
