// Counts the algorithmic floating-point operations of the device pair
// arithmetic (paper_1709_02410_amd/csrc/pair_math.h), compiled for the CPU
// with a counting scalar type.  Rule: fused multiply-add = 2, add, subtract
// and multiply = 1, reciprocal square root = 1, negation, comparison and
// selection = 0.  An operation is counted only when one of its operands
// depends on the source blob of the pair: operations on the target blob
// alone (or on constants) are done once per target by the kernels, not once
// per pair.  Precision bookkeeping of the FP32 path (low parts of the
// positions, compensated sums) is not part of the formula and is not counted.
//
// Prints one JSON object:
//   shared      geometry and coefficients of one pair (the three coordinate
//               differences included), far branch (r > 2a)
//   apply       one application M_ij f_j accumulated into a sum
//   block       the 3 x 3 block M_ij written out from the coefficients
//   block_apply one right-hand side contracted with the written-out block
//   vjp_pair    one unordered pair of the symmetric VJP: the analytic pair
//               gradient, both blobs' gradient sums and the four products
//               (two per blob)
//   vjp_self    one ordered pair seen from the target only (the self pair,
//               or every pair of the non-symmetric VJP kernel)
#include <cmath>
#include <cstdio>

struct Flop {
    double v;
    bool p;  // depends on the source blob
    Flop() : v(0.0), p(false) {}
    Flop(double x) : v(x), p(false) {}
};

static long g_count = 0;

static Flop counted(double v, bool p, int n) {
    if (p) g_count += n;
    Flop f(v);
    f.p = p;
    return f;
}
inline Flop operator+(Flop a, Flop b) { return counted(a.v + b.v, a.p || b.p, 1); }
inline Flop operator-(Flop a, Flop b) { return counted(a.v - b.v, a.p || b.p, 1); }
inline Flop operator*(Flop a, Flop b) { return counted(a.v * b.v, a.p || b.p, 1); }
inline Flop operator-(Flop a) {
    Flop f(-a.v);
    f.p = a.p;
    return f;
}
inline Flop& operator+=(Flop& a, Flop b) { return a = a + b; }
inline bool operator<=(Flop a, Flop b) { return a.v <= b.v; }
inline bool operator<(Flop a, Flop b) { return a.v < b.v; }
inline bool operator>(Flop a, Flop b) { return a.v > b.v; }
inline bool operator>=(Flop a, Flop b) { return a.v >= b.v; }
inline bool operator==(Flop a, Flop b) { return a.v == b.v; }
inline Flop fma_(Flop a, Flop b, Flop c) { return counted(a.v * b.v + c.v, a.p || b.p || c.p, 2); }
inline void issue_together(Flop&, Flop&) {}

#include "../../paper_1709_02410_amd/csrc/pair_math.h"

namespace rpyw {
template <>
inline Flop rsq<Flop>(Flop x) {
    return counted(1.0 / std::sqrt(x.v), x.p, 1);
}
}  // namespace rpyw

using namespace rpyw;

static Flop src(double v) {
    Flop f(v);
    f.p = true;
    return f;
}

int main() {
    // a far pair (r > 2): target at (1, 2, 3), source at (6, -1, 2)
    const Flop xi(1.0), yi(2.0), zi(3.0);
    const Flop xj = src(6.0), yj = src(-1.0), zj = src(2.0);
    const Flop fi[3] = {Flop(0.3), Flop(-0.2), Flop(0.7)};
    const Flop gi[3] = {Flop(-0.4), Flop(0.9), Flop(0.1)};
    const Flop fj[3] = {src(0.5), src(0.1), src(-0.6)};
    const Flop gj[3] = {src(0.2), src(-0.8), src(0.4)};

    g_count = 0;
    const Flop dx = xi - xj, dy = yi - yj, dz = zi - zj;
    PairPre<Flop> pre = pair_pre<Flop>(pair_geo<Flop>(dx, dy, dz, zi, zj), dz, zi, zj);
    if (pair_near(pre)) pair_fix(pre);
    PairCoef<Flop> c = pair_fin(pre);
    const long shared = g_count;

    g_count = 0;
    Flop u[3];
    pair_apply<Flop>(c, dx, dy, dz, fj[0], fj[1], fj[2], u[0], u[1], u[2]);
    const long apply = g_count;

    g_count = 0;
    const PairBlock<Flop> m = pair_block<Flop>(c, dx, dy, dz);
    const long block = g_count;
    g_count = 0;
    Flop v[3];
    block_apply<Flop>(m, fj[0], fj[1], fj[2], v[0], v[1], v[2]);
    const long block_apply_n = g_count;

    // symmetric VJP, one unordered pair: target side and source side
    g_count = 0;
    PairCoef<Flop> p;
    const PairGrad<Flop> g = pair_grad<Flop>(dx, dy, dz, zi, zj, gi, fj, fi, gj, &p);
    Flop acc[9], sacc[9];
    acc[0] += g.dx;
    acc[1] += g.dy;
    acc[2] += fma_(zj, g.zz, g.dz + g.rz);
    pair_apply<Flop>(p, dx, dy, dz, fj[0], fj[1], fj[2], acc[3], acc[4], acc[5]);
    pair_apply<Flop>(p, dx, dy, dz, gj[0], gj[1], gj[2], acc[6], acc[7], acc[8]);
    const long vjp_self = g_count + 3;  // + the three coordinate differences
    sacc[0] = sacc[0] - g.dx;
    sacc[1] = sacc[1] - g.dy;
    sacc[2] += fma_(zi, g.zz, g.rz - g.dz);
    const Flop t = p.kcp;
    p.kcp = p.kcm;
    p.kcm = t;
    pair_apply<Flop>(p, dx, dy, dz, fi[0], fi[1], fi[2], sacc[3], sacc[4], sacc[5]);
    pair_apply<Flop>(p, dx, dy, dz, gi[0], gi[1], gi[2], sacc[6], sacc[7], sacc[8]);
    const long vjp_pair = g_count + 3;

    std::printf(
        "{\"shared\": %ld, \"apply\": %ld, \"block\": %ld, \"block_apply\": %ld, \"vjp_pair\": %ld, "
        "\"vjp_self\": %ld}\n",
        shared, apply, block, block_apply_n, vjp_pair, vjp_self);
    return 0;
}
