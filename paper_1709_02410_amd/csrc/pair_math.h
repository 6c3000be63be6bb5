// Device-side pair arithmetic of the wall-corrected RPY blob mobility
// (arXiv:1709.02410, Sec. II.A: Rotne-Prager-Yamakawa blocks with the
// no-slip wall correction of the Rotne-Prager-Blake tensor; Sec. IV opening:
// overlap regularisations keeping M SPD).
//
// Everything here works in units where the blob radius is 1 and M is measured
// in mu0 = 1/(6 pi eta a): positions arrive pre-divided by a with heights
// already regularised (z~ = max(z, a)), forces arrive pre-multiplied by
// B = min(z/a, 1), and the caller multiplies sums by mu0 * B_target.
//
// Notation per pair (target i, source j):
//   d = r~_i - r~_j = (dx, dy, dz), r2 = |d|^2          (free RPY part)
//   R = r~_i - mirror(r~_j) = (dx, dy, Rz), Rz = z_i + z_j, R2 = |R|^2
//   w = 1/|R|, X = w^2, zz = z_i z_j                      (image part)
// The wall correction, written in q = Rz w, p = z_j w, s = X, is rearranged
// as polynomials in X whose coefficients depend on u = Rz^2 X and v = zz X:
//   |R| A  = -3/4 - 3/2 v + X(-1/2 + 3/2 u + X(1/2 - 5/2 u))
//   |R| B  = -3/4 + 9/2 v + X( 3/2 - 15/2 u + X(-5/2 + 35/2 u))
//   |R| C  = -3/4 dz + Rz g,   |R| C' = -3/4 dz - Rz g,   g = 5 X^2 - 3/4 - |R| B
//   |R| E  = -u |R| B - 3/4 - 3/2 u + 3/2 v + X(-1/2 - 3/2 u + X(-3/2 + 25/2 u))
// (using q p - p^2 = zz X, the identity that removes p).  The block acts as
//   (Mf)_x = (c1 + w A') f_x + dx [c2 (d.f) + w X (B' G + C' f_z)]   (same y)
//   (Mf)_z = (c1 + w E') f_z + c2 (d.f) dz + w X (Cm' G)
// with G = dx f_x + dy f_y and primes denoting the |R|-scaled coefficients;
// the free RPY coefficients are c1, c2 with c2 already divided by r2:
//   r > 2: c1 = 3/(4r) + 1/(2r^3),  c2 = 3/(4r^3) - 3/(2r^5)
//   r <= 2: c1 = 1 - 9r/32,          c2 = 3/(32 r);   r = 0: c1 = 1, c2 = 0.
#pragma once

#include <hip/hip_runtime.h>

namespace rpyw {

// Fused multiply-add in the precision of the operands.
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Round to the nearest integer, ties to even.
__device__ __forceinline__ float rint_(float x) { return __builtin_rintf(x); }
__device__ __forceinline__ double rint_(double x) { return __builtin_rint(x); }

template <typename R>
__device__ __forceinline__ R rsq(R x);

// An empty asm statement that takes both values as inputs and outputs: every
// use of either is scheduled after both are computed (used to issue two
// reciprocal square roots back to back, so that their latencies overlap).
template <typename R>
__device__ __forceinline__ void issue_together(R& a, R& b) {
    __asm__ volatile("" : "+v"(a), "+v"(b));
}

// FP32: the hardware reciprocal square root (about 1 ulp).
template <>
__device__ __forceinline__ float rsq<float>(float x) {
    return __builtin_amdgcn_rsqf(x);
}

// FP64: hardware estimate refined by one third-order (Householder) step,
// y <- y + y e (1/2 + 3/8 e) with e = 1 - x y^2, which triples the number of
// correct bits of the estimate.
template <>
__device__ __forceinline__ double rsq<double>(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// Geometry shared by every right-hand side of one pair.
template <typename R>
struct PairCoef {
    R c1;   // free identity coefficient
    R c2;   // free d d^T coefficient (divided by r2)
    R cc;   // c1 + w |R|A   (in-plane diagonal)
    R cz;   // c1 + w |R|E   (normal diagonal)
    R kb;   // w X |R|B
    R kcp;  // w X |R|C      (in-plane velocity from normal force)
    R kcm;  // w X |R|C'     (normal velocity from in-plane force)
};

// The pair coefficients in three stages, so that several pairs can share one
// overlap branch.  pair_pre evaluates everything with the far-field free
// coefficients (r > 2); pair_fix replaces c1, c2 where r <= 2 (the guard
// keeps r = 0 finite: c1 = 1, c2 d = 0); pair_fin forms the two diagonal
// coefficients.  dx, dy, dz: target minus source; zi, zj: regularised
// heights.
template <typename R>
struct PairPre {
    R c1, c2, w, rA, rE, kb, kcp, kcm, r2;
};

// The two distances of a pair and their reciprocal square roots, the first
// stage of pair_pre (kept separate so that callers can issue the reciprocal
// square roots of several pairs before any of their results is used).
template <typename R>
struct PairGeo {
    R rz, rz2, r2, w, ir;
};

template <typename R>
__device__ __forceinline__ PairGeo<R> pair_geo(R dx, R dy, R dz, R zi, R zj) {
    PairGeo<R> g;
    g.rz = zi + zj;
    const R h2 = fma_(dy, dy, dx * dx);
    g.r2 = fma_(dz, dz, h2);
    g.rz2 = g.rz * g.rz;
    g.w = rsq<R>(h2 + g.rz2);
    g.ir = rsq<R>(g.r2);
    return g;
}

template <typename R>
__device__ __forceinline__ PairPre<R> pair_pre(const PairGeo<R>& gm, R dz, R zi, R zj) {
    PairPre<R> o;
    const R rz = gm.rz, rz2 = gm.rz2, r2 = gm.r2, w = gm.w;
    const R X = w * w;
    const R wX = w * X;
    // free RPY, far branch (r > 2)
    const R ir = gm.ir;
    const R ir2 = ir * ir;
    o.c1 = ir * fma_(ir2, R(0.5), R(0.75));
    o.c2 = (ir * ir2) * fma_(ir2, R(-1.5), R(0.75));
    const R u = rz2 * X;
    // v = zz X enters only as v c; written (z_j X)(c z_i) so that c z_i is
    // hoisted out of loops over sources.
    const R zjX = zj * X;
    o.rA = fma_(X, fma_(X, fma_(u, R(-2.5), R(0.5)), fma_(u, R(1.5), R(-0.5))), fma_(zjX, R(-1.5) * zi, R(-0.75)));
    const R rB =
        fma_(X, fma_(X, fma_(u, R(17.5), R(-2.5)), fma_(u, R(-7.5), R(1.5))), fma_(zjX, R(4.5) * zi, R(-0.75)));
    const R g = fma_(X * X, R(5.0), R(-0.75)) - rB;
    const R cw = dz * R(-0.75);
    const R qE = fma_(X, fma_(X, fma_(u, R(12.5), R(-1.5)), fma_(u, R(-1.5), R(-0.5))),
                      fma_(zjX, R(1.5) * zi, fma_(u, R(-1.5), R(-0.75))));
    o.rE = fma_(-u, rB, qE);
    o.w = w;
    o.kb = wX * rB;
    o.kcp = wX * fma_(rz, g, cw);
    o.kcm = wX * fma_(-rz, g, cw);
    o.r2 = r2;
    return o;
}

template <typename R>
__device__ __forceinline__ PairPre<R> pair_pre(R dx, R dy, R dz, R zi, R zj) {
    return pair_pre<R>(pair_geo<R>(dx, dy, dz, zi, zj), dz, zi, zj);
}

template <typename R>
__device__ __forceinline__ bool pair_near(const PairPre<R>& p) {
    return p.r2 <= R(4);
}

template <typename R>
__device__ __forceinline__ void pair_fix(PairPre<R>& p) {
    const bool near = pair_near(p);
    const R irg = rsq<R>(p.r2 > R(1e-30) ? p.r2 : R(1e-30));
    const R c1n = fma_(R(-9.0 / 32.0), p.r2 * irg, R(1));
    const R c2n = R(3.0 / 32.0) * irg;
    p.c1 = near ? c1n : p.c1;
    p.c2 = near ? c2n : p.c2;
}

template <typename R>
__device__ __forceinline__ PairCoef<R> pair_fin(const PairPre<R>& p) {
    PairCoef<R> o;
    o.c1 = p.c1;
    o.c2 = p.c2;
    o.cc = fma_(p.w, p.rA, p.c1);
    o.cz = fma_(p.w, p.rE, p.c1);
    o.kb = p.kb;
    o.kcp = p.kcp;
    o.kcm = p.kcm;
    return o;
}

// One pair with its own overlap branch: entered by the whole wave when any
// lane has an overlapping pair (rare: self pairs and touching neighbours).
template <typename R>
__device__ __forceinline__ PairCoef<R> pair_coef(R dx, R dy, R dz, R zi, R zj) {
    PairPre<R> p = pair_pre<R>(dx, dy, dz, zi, zj);
    if (__builtin_amdgcn_ballot_w64(pair_near(p))) {
        __asm__ volatile("" ::: "memory");  // keep this a branch: do not speculate it
        pair_fix(p);
    }
    return pair_fin(p);
}

// Accumulate M_ij f_j (units of mu0, B factors excluded) into (ux, uy, uz).
template <typename R>
__device__ __forceinline__ void pair_apply(const PairCoef<R>& p, R dx, R dy, R dz, R fx, R fy, R fz, R& ux,
                                           R& uy, R& uz) {
    const R G = fma_(dy, fy, dx * fx);
    const R D = fma_(dz, fz, G);
    const R t0 = p.c2 * D;
    const R t = fma_(p.kcp, fz, fma_(p.kb, G, t0));
    ux = fma_(t, dx, fma_(p.cc, fx, ux));
    uy = fma_(t, dy, fma_(p.cc, fy, uy));
    uz = fma_(t0, dz, fma_(p.kcm, G, fma_(p.cz, fz, uz)));
}

// The 3 x 3 block M_ij that pair_apply applies (units of mu0, B factors
// excluded), written out for contracting one pair with a block of
// right-hand sides.  From pair_apply: t = (kb + c2) (dx fx + dy fy) +
// (kcp + c2 dz) fz enters along (dx, dy), and the normal row is
// cz fz + (kcm + c2 dz)(dx fx + dy fy) + c2 dz^2 fz.  The block is not
// symmetric (in-plane force to normal velocity and back have different wall
// coefficients), but M_xy = M_yx.
template <typename R>
struct PairBlock {
    R xx, xy, xz, yy, yz, zx, zy, zz;
};

template <typename R>
__device__ __forceinline__ PairBlock<R> pair_block(const PairCoef<R>& p, R dx, R dy, R dz) {
    PairBlock<R> m;
    const R qb = p.kb + p.c2;
    const R qx = qb * dx;
    m.xx = fma_(qx, dx, p.cc);
    m.xy = qx * dy;
    m.yy = fma_(qb * dy, dy, p.cc);
    const R pz = fma_(p.c2, dz, p.kcp);
    m.xz = dx * pz;
    m.yz = dy * pz;
    const R qz = fma_(p.c2, dz, p.kcm);
    m.zx = dx * qz;
    m.zy = dy * qz;
    m.zz = fma_(p.c2 * dz, dz, p.cz);
    return m;
}

// u += M f for one right-hand side: the contraction that the matrix cores
// carry out for a block of right-hand sides (this form serves the host
// checks and the operation count).
template <typename R>
__device__ __forceinline__ void block_apply(const PairBlock<R>& m, R fx, R fy, R fz, R& ux, R& uy, R& uz) {
    ux = fma_(m.xx, fx, fma_(m.xy, fy, fma_(m.xz, fz, ux)));
    uy = fma_(m.xy, fx, fma_(m.yy, fy, fma_(m.yz, fz, uy)));
    uz = fma_(m.zx, fx, fma_(m.zy, fy, fma_(m.zz, fz, uz)));
}

// Gradient of Phi = a^T M b + a2^T M b2 (units of mu0, radius 1) for one
// pair, with respect to the base variables of the pair geometry
// (dx, dy, dz, Rz = z_i + z_j, zz = z_i z_j).  Writing
//   a^T M b = c1 (a.b) + c2 D_a D_b
//           + w [|R|A h_ab + X |R|B G_a G_b + X Cw (G_a b_z + a_z G_b)
//                + X Vw (G_a b_z - a_z G_b) + |R|E a_z b_z],
// G_v = dx v_x + dy v_y, D_v = G_v + dz v_z, h_ab = a_x b_x + a_y b_y,
// Cw = -3/4 dz, Vw = Rz X Pv, the two forms share all coefficients and
// enter through the sums S1, S2, SA, SB, SC, SV, SE below.  w and X depend
// on R2 = dx^2 + dy^2 + Rz^2 only, c1 and c2 on r2 = dx^2 + dy^2 + dz^2.
// Target derivatives: d/dx_i = g.dx, d/dy_i = g.dy,
//   d/dz_i = g.dz + g.rz + z_j g.zz;  source: d/dx_j = -g.dx,
//   d/dz_j = -g.dz + g.rz + z_i g.zz.  Coincident blobs (r2 = 0) give no
// free-part derivative.  Also returns the pair coefficients for value sums.
template <typename R>
struct PairGrad {
    R dx, dy, dz, rz, zz;
};

template <typename R>
__device__ __forceinline__ PairGrad<R> pair_grad(R dx, R dy, R dz, R zi, R zj, const R* a, const R* b,
                                                 const R* a2, const R* b2, PairCoef<R>* coef) {
    const R rz = zi + zj;
    const R h2 = fma_(dy, dy, dx * dx);
    const R r2 = fma_(dz, dz, h2);
    const R rz2 = rz * rz;
    const R R2 = h2 + rz2;
    R w = rsq<R>(R2);
    R ir = rsq<R>(r2);
    issue_together(w, ir);
    const R X = w * w;
    const R wX = w * X;
    // free RPY coefficients and their derivatives in r2
    const R ir2 = ir * ir;
    const R ir3 = ir * ir2;
    R c1 = ir * fma_(ir2, R(0.5), R(0.75));
    R c2 = ir3 * fma_(ir2, R(-1.5), R(0.75));
    R dc1 = -ir3 * fma_(ir2, R(0.75), R(0.375));
    R dc2 = ir3 * ir2 * fma_(ir2, R(3.75), R(-1.125));
    const bool near = r2 <= R(4);
    if (__builtin_amdgcn_ballot_w64(near)) {
        __asm__ volatile("" ::: "memory");
        const R irg = rsq<R>(r2 > R(1e-30) ? r2 : R(1e-30));
        const bool zero = r2 == R(0);
        c1 = near ? fma_(R(-9.0 / 32.0), r2 * irg, R(1)) : c1;
        c2 = near ? R(3.0 / 32.0) * irg : c2;
        dc1 = near ? (zero ? R(0) : R(-9.0 / 64.0) * irg) : dc1;
        dc2 = near ? (zero ? R(0) : R(-3.0 / 64.0) * irg * irg * irg) : dc2;
    }
    // bilinear building blocks
    const R Ga = fma_(dy, a[1], dx * a[0]), Gb = fma_(dy, b[1], dx * b[0]);
    const R Gc = fma_(dy, a2[1], dx * a2[0]), Gd = fma_(dy, b2[1], dx * b2[0]);
    const R Da = fma_(dz, a[2], Ga), Db = fma_(dz, b[2], Gb);
    const R Dc = fma_(dz, a2[2], Gc), Dd = fma_(dz, b2[2], Gd);
    const R SA = fma_(a[0], b[0], a[1] * b[1]) + fma_(a2[0], b2[0], a2[1] * b2[1]);
    const R SE = fma_(a[2], b[2], a2[2] * b2[2]);
    const R S1 = SA + SE;
    const R S2 = fma_(Da, Db, Dc * Dd);
    const R SB = fma_(Ga, Gb, Gc * Gd);
    const R SC = fma_(Ga, b[2], a[2] * Gb) + fma_(Gc, b2[2], a2[2] * Gd);
    const R SV = fma_(Ga, b[2], -a[2] * Gb) + fma_(Gc, b2[2], -a2[2] * Gd);
    // their derivatives in dx, dy, dz
    const R S2x = fma_(a[0], Db, Da * b[0]) + fma_(a2[0], Dd, Dc * b2[0]);
    const R S2y = fma_(a[1], Db, Da * b[1]) + fma_(a2[1], Dd, Dc * b2[1]);
    const R S2z = fma_(a[2], Db, Da * b[2]) + fma_(a2[2], Dd, Dc * b2[2]);
    const R SBx = fma_(a[0], Gb, Ga * b[0]) + fma_(a2[0], Gd, Gc * b2[0]);
    const R SBy = fma_(a[1], Gb, Ga * b[1]) + fma_(a2[1], Gd, Gc * b2[1]);
    const R SCx = fma_(a[0], b[2], a[2] * b[0]) + fma_(a2[0], b2[2], a2[2] * b2[0]);
    const R SCy = fma_(a[1], b[2], a[2] * b[1]) + fma_(a2[1], b2[2], a2[2] * b2[1]);
    const R SVx = fma_(a[0], b[2], -a[2] * b[0]) + fma_(a2[0], b2[2], -a2[2] * b2[0]);
    const R SVy = fma_(a[1], b[2], -a[2] * b[1]) + fma_(a2[1], b2[2], -a2[2] * b2[1]);
    // wall coefficients and their partial derivatives in X, Rz, zz
    const R zz = zi * zj;
    const R a1 = fma_(zz, R(-1.5), R(-0.5)), a2c = fma_(rz2, R(1.5), R(0.5)), a3 = rz2 * R(-2.5);
    const R rA = fma_(X, fma_(X, fma_(X, a3, a2c), a1), R(-0.75));
    const R rA_X = fma_(X, fma_(X, R(3) * a3, R(2) * a2c), a1);
    const R rA_rz = X * X * rz * fma_(X, R(-5), R(3));
    const R rA_zz = R(-1.5) * X;
    const R b1 = fma_(zz, R(4.5), R(1.5)), b2c = fma_(rz2, R(-7.5), R(-2.5)), b3 = rz2 * R(17.5);
    const R rB = fma_(X, fma_(X, fma_(X, b3, b2c), b1), R(-0.75));
    const R rB_X = fma_(X, fma_(X, R(3) * b3, R(2) * b2c), b1);
    const R rB_rz = X * X * rz * fma_(X, R(35), R(-15));
    const R rB_zz = R(4.5) * X;
    const R v2 = fma_(rz2, R(7.5), R(7.5));
    const R pv = fma_(X, fma_(-X, b3, v2), -b1);
    const R vw = (rz * X) * pv;
    const R vw_X = rz * fma_(X, fma_(X, R(-3) * b3, R(2) * v2), -b1);
    const R vw_rz = fma_(X * X * rz2, fma_(X, R(-35), R(15)), X * pv);
    const R vw_zz = R(-4.5) * rz * X;
    const R cw = dz * R(-0.75);
    const R e1 = fma_(zz, R(1.5), fma_(rz2, R(-0.75), R(-0.5)));
    const R e2 = fma_(rz2, fma_(zz, R(-4.5), R(-3.0)), R(-1.5));
    const R e3 = rz2 * fma_(rz2, R(7.5), R(15.0));
    const R e4 = (rz2 * rz2) * R(-17.5);
    const R rE = fma_(X, fma_(X, fma_(X, fma_(X, e4, e3), e2), e1), R(-0.75));
    const R rE_X = fma_(X, fma_(X, fma_(X, R(4) * e4, R(3) * e3), R(2) * e2), e1);
    const R de1 = R(-1.5) * rz;
    const R de2 = R(2) * rz * fma_(zz, R(-4.5), R(-3.0));
    const R de3 = R(30) * rz * (rz2 + R(1));
    const R de4 = R(-70) * rz * rz2;
    const R rE_rz = X * fma_(X, fma_(X, fma_(X, de4, de3), de2), de1);
    const R rE_zz = X * fma_(X, R(-4.5) * rz2, R(1.5));
    // Phi = c1 S1 + c2 S2 + w P1 + w X P2
    const R P1 = fma_(rA, SA, rE * SE);
    const R P2 = fma_(rB, SB, fma_(cw, SC, vw * SV));
    const R P1_X = fma_(rA_X, SA, rE_X * SE);
    const R P2_X = fma_(rB_X, SB, vw_X * SV);
    const R dR2 = -wX * fma_(X * X, P2_X, fma_(X, fma_(R(1.5), P2, P1_X), R(0.5) * P1));
    const R dr2 = fma_(dc1, S1, dc2 * S2);
    const R sh = R(2) * (dr2 + dR2);
    PairGrad<R> g;
    g.dx = fma_(sh, dx, fma_(c2, S2x, wX * fma_(rB, SBx, fma_(cw, SCx, vw * SVx))));
    g.dy = fma_(sh, dy, fma_(c2, S2y, wX * fma_(rB, SBy, fma_(cw, SCy, vw * SVy))));
    g.dz = fma_(R(2) * dr2, dz, fma_(c2, S2z, wX * R(-0.75) * SC));
    g.rz = fma_(R(2) * dR2, rz, fma_(w, fma_(rA_rz, SA, rE_rz * SE), wX * fma_(rB_rz, SB, vw_rz * SV)));
    g.zz = fma_(w, fma_(rA_zz, SA, rE_zz * SE), wX * fma_(rB_zz, SB, vw_zz * SV));
    if (coef) {
        coef->c1 = c1;
        coef->c2 = c2;
        coef->cc = fma_(w, rA, c1);
        coef->cz = fma_(w, rE, c1);
        coef->kb = wX * rB;
        coef->kcp = wX * (cw + vw);
        coef->kcm = wX * (cw - vw);
    }
    return g;
}

// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest, no reassociation).
template <typename R>
__device__ __forceinline__ void two_sum_acc(R& hi, R& lo, R b) {
    const R s = hi + b;
    const R bp = s - hi;
    const R ap = s - bp;
    lo += (hi - ap) + (b - bp);
    hi = s;
}

}  // namespace rpyw
