// Derivatives of u = M(r) f (arXiv:1709.02410, Sec. III: derivatives of the
// blob mobility produce the thermal drift that random finite differences
// estimate).
//
// Vector-Jacobian product for L = sum_k g_k . u_k.  With F~ = B f and
// G~ = B g (B = min(z/a, 1)) and Mhat the unregularised-height block,
//   dL/dr~_k = mu0 sum_j d1[G~_k^T Mhat(r~_k, r~_j) F~_j + F~_k^T Mhat(r~_k, r~_j) G~_j]
// (reciprocity turns the source-side appearance of r_k into the second
// form; the j = k term is then the total derivative of the self block), and
//   dL/dB_k = mu0 (g_k . (Mhat F~)_k + f_k . (Mhat G~)_k),  grad_f = mu0 B (Mhat G~).
// One fused pass per target evaluates the analytic pair gradient
// (pair_grad) and the two products; the epilogue applies the chain rule of
// the regularisation: d r~/dz = 1{z >= a}, dB/dz = 1{z < a}/a.
#include <algorithm>

#include "pair_math.h"
#include "records.h"
#include "rpyw_internal.h"
#include "sym_pairs.h"

namespace rpyw {

namespace {

constexpr int kQ = 9;  // grad (3), Mhat F~ (3), Mhat G~ (3)

template <typename R, int TILE>
__global__ __launch_bounds__(kBlock) void vjp_kernel(const R* __restrict__ rec, int64_t N, int splits,
                                                     int64_t chunk, double* __restrict__ part) {
    constexpr int RW = rec_w<R, 2>();
    constexpr int PW = pos_slots<R>();
    __shared__ __attribute__((aligned(16))) R tile[TILE * RW];
    const int b = blockIdx.x;
    const int split = b % splits;
    const int64_t first = (int64_t)(b / splits) * kBlock;
    const int64_t s0 = (int64_t)split * chunk;
    const int64_t s1 = s0 + chunk < N ? s0 + chunk : N;
    const int64_t i = first + threadIdx.x;
    const R* me = rec + (i < N ? i : N - 1) * RW;
    const R x = me[0], y = me[1], z = me[2];
    R xl = R(0), yl = R(0);
    if constexpr (sizeof(R) == 4) {
        xl = me[3];
        yl = me[4];
    }
    const R A[3] = {me[PW + 3], me[PW + 4], me[PW + 5]};   // G~ of the target
    const R A2[3] = {me[PW], me[PW + 1], me[PW + 2]};      // F~ of the target
    R acc[kQ], hi[kQ], lo[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = hi[q] = lo[q] = R(0);
    for (int64_t t0 = s0; t0 < s1; t0 += TILE) {
        const int n = (int)((s1 - t0) < TILE ? (s1 - t0) : TILE);
        __syncthreads();
        const R* g = rec + t0 * RW;
        for (int e = threadIdx.x; e < n * RW; e += kBlock) tile[e] = g[e];
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            const R* s = tile + j * RW;
            R dx = x - s[0], dy = y - s[1];
            if constexpr (sizeof(R) == 4) {
                dx += xl - s[3];
                dy += yl - s[4];
            }
            const R dz = z - s[2];
            const R Bf[3] = {s[PW], s[PW + 1], s[PW + 2]};       // F~ of the source
            const R Bg[3] = {s[PW + 3], s[PW + 4], s[PW + 5]};   // G~ of the source
            PairCoef<R> c;
            const PairGrad<R> gr = pair_grad<R>(dx, dy, dz, z, s[2], A, Bf, A2, Bg, &c);
            acc[0] += gr.dx;
            acc[1] += gr.dy;
            acc[2] += fma_(s[2], gr.zz, gr.dz + gr.rz);
            pair_apply<R>(c, dx, dy, dz, Bf[0], Bf[1], Bf[2], acc[3], acc[4], acc[5]);
            pair_apply<R>(c, dx, dy, dz, Bg[0], Bg[1], Bg[2], acc[6], acc[7], acc[8]);
        }
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                two_sum_acc(hi[q], lo[q], acc[q]);
                acc[q] = R(0);
            }
        }
    }
    if (i >= N) return;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const double v = sizeof(R) == 4 ? (double)hi[q] + (double)lo[q] : (double)acc[q];
        part[((int64_t)split * kQ + q) * N + i] = v;
    }
}

__global__ void vjp_epilogue(const double* __restrict__ part, const double* __restrict__ pos,
                             const double* __restrict__ f, const double* __restrict__ g, int64_t N, int splits,
                             double inv_a, double mu0, double* __restrict__ grad_pos, double* __restrict__ grad_f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s[kQ];
    for (int q = 0; q < kQ; ++q) {
        double t = 0.0;
        for (int p = 0; p < splits; ++p) t += part[((int64_t)p * kQ + q) * N + i];
        s[q] = t;
    }
    const double z = pos[3 * i + 2] * inv_a;
    const double B = z < 1.0 ? z : 1.0;
    if (grad_pos) {
        const double dLdB = mu0 * (g[3 * i] * s[3] + g[3 * i + 1] * s[4] + g[3 * i + 2] * s[5] + f[3 * i] * s[6] +
                                   f[3 * i + 1] * s[7] + f[3 * i + 2] * s[8]);
        grad_pos[3 * i] = mu0 * inv_a * s[0];
        grad_pos[3 * i + 1] = mu0 * inv_a * s[1];
        grad_pos[3 * i + 2] = z < 1.0 ? inv_a * dLdB : mu0 * inv_a * s[2];
    }
    if (grad_f)
        for (int c = 0; c < 3; ++c) grad_f[3 * i + c] = mu0 * B * s[6 + c];
}

// Symmetric VJP (sym_pairs.h).  For the pair (i, j) the scalar
//   Phi = G~_i^T Mhat(r~_i, r~_j) F~_j + F~_i^T Mhat(r~_i, r~_j) G~_j
// is also the pair's term seen from j (reciprocity), so one analytic pair
// gradient gives both blobs' contributions: the target derivatives for i and
// the source derivatives for j.  The two products are applied directly for i
// and transposed (wall coefficients exchanged) for j.
template <typename R>
struct VjpBody {
    static constexpr int KREC = 2;  // F~, G~
    static constexpr int NQ = kQ;   // grad (3), Mhat F~ (3), Mhat G~ (3)
    static constexpr int kUnroll = 4;
    static constexpr bool kDuo = false;
    template <bool SYM>
    __device__ static void pair(const SymTarget<R, 2>& t, const R* r, R (&acc)[kQ], R (&src)[kQ], const Box<R>&) {
        constexpr int PW = pos_slots<R>();
        R dx, dy, dz;
        sym_diff(t, r, dx, dy, dz);
        const R zj = r[2];
        const R Bf[3] = {r[PW], r[PW + 1], r[PW + 2]};
        const R Bg[3] = {r[PW + 3], r[PW + 4], r[PW + 5]};
        PairCoef<R> p;
        const PairGrad<R> g = pair_grad<R>(dx, dy, dz, t.z, zj, t.f[1], Bf, t.f[0], Bg, &p);
        acc[0] += g.dx;
        acc[1] += g.dy;
        acc[2] += fma_(zj, g.zz, g.dz + g.rz);
        pair_apply<R>(p, dx, dy, dz, Bf[0], Bf[1], Bf[2], acc[3], acc[4], acc[5]);
        pair_apply<R>(p, dx, dy, dz, Bg[0], Bg[1], Bg[2], acc[6], acc[7], acc[8]);
        if constexpr (SYM) {
            src[0] = -g.dx;
            src[1] = -g.dy;
            src[2] = fma_(t.z, g.zz, g.rz - g.dz);
            const R x = p.kcp;
            p.kcp = p.kcm;
            p.kcm = x;
#pragma unroll
            for (int q = 3; q < kQ; ++q) src[q] = R(0);
            pair_apply<R>(p, dx, dy, dz, t.f[0][0], t.f[0][1], t.f[0][2], src[3], src[4], src[5]);
            pair_apply<R>(p, dx, dy, dz, t.f[1][0], t.f[1][1], t.f[1][2], src[6], src[7], src[8]);
        }
    }
};

template <typename R>
__global__ void sym_vjp_epilogue(const double* __restrict__ tpart, const R* __restrict__ spart,
                                 const double* __restrict__ pos, const double* __restrict__ f,
                                 const double* __restrict__ g, int64_t N, int ng, int C, int Hmax, int G,
                                 double inv_a, double mu0, double* __restrict__ grad_pos, double* __restrict__ grad_f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s[kQ];
    for (int q = 0; q < kQ; ++q) s[q] = sym_gather<R>(tpart, spart, i, ng, C, Hmax, kQ, q, G);
    const double z = pos[3 * i + 2] * inv_a;
    const double B = z < 1.0 ? z : 1.0;
    if (grad_pos) {
        const double dLdB = mu0 * (g[3 * i] * s[3] + g[3 * i + 1] * s[4] + g[3 * i + 2] * s[5] + f[3 * i] * s[6] +
                                   f[3 * i + 1] * s[7] + f[3 * i + 2] * s[8]);
        grad_pos[3 * i] = mu0 * inv_a * s[0];
        grad_pos[3 * i + 1] = mu0 * inv_a * s[1];
        grad_pos[3 * i + 2] = z < 1.0 ? inv_a * dLdB : mu0 * inv_a * s[2];
    }
    if (grad_f)
        for (int c = 0; c < 3; ++c) grad_f[3 * i + c] = mu0 * B * s[6 + c];
}

// div_i,a = sum_j sum_b d(M_ij)_ab / d r_j,b (source derivative; for j = i
// the total derivative of the self block).  One wave per target: lane l takes
// the sources j = l (mod 64), and the 64 lane sums are added in lane order,
// so the result does not depend on scheduling.  Meant for the small systems
// on which the divergence is checked (every pair costs nine gradient
// evaluations).
template <typename R>
__global__ __launch_bounds__(64) void divergence_kernel(const double* __restrict__ pos, int64_t N, double inv_a,
                                                        double mu0, double* __restrict__ div) {
    __shared__ double red[3][64];
    const int64_t i = blockIdx.x;
    const int l = threadIdx.x;
    const double xi = pos[3 * i] * inv_a, yi = pos[3 * i + 1] * inv_a, zri = pos[3 * i + 2] * inv_a;
    const double Bi = zri < 1.0 ? zri : 1.0, zti = zri < 1.0 ? 1.0 : zri;
    const double dBi = zri < 1.0 ? 1.0 : 0.0, dzti = zri < 1.0 ? 0.0 : 1.0;
    const R zero[3] = {R(0), R(0), R(0)};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t j = l; j < N; j += 64) {
        const double xj = pos[3 * j] * inv_a, yj = pos[3 * j + 1] * inv_a, zrj = pos[3 * j + 2] * inv_a;
        const double Bj = zrj < 1.0 ? zrj : 1.0, ztj = zrj < 1.0 ? 1.0 : zrj;
        const double dBj = zrj < 1.0 ? 1.0 : 0.0, dztj = zrj < 1.0 ? 0.0 : 1.0;
        const R dx = (R)(xi - xj), dy = (R)(yi - yj), dz = (R)(zti - ztj);
        for (int a = 0; a < 3; ++a) {
            const R ea[3] = {R(a == 0), R(a == 1), R(a == 2)};
            for (int b = 0; b < 3; ++b) {
                const R eb[3] = {R(b == 0), R(b == 1), R(b == 2)};
                PairCoef<R> c;
                const PairGrad<R> g = pair_grad<R>(dx, dy, dz, (R)zti, (R)ztj, ea, eb, zero, zero, &c);
                R u[3] = {R(0), R(0), R(0)};
                pair_apply<R>(c, dx, dy, dz, eb[0], eb[1], eb[2], u[0], u[1], u[2]);
                const double phi = (double)u[a];
                double d = 0.0;
                if (j != i) {
                    if (b == 0)
                        d = -(double)g.dx * Bi * Bj;
                    else if (b == 1)
                        d = -(double)g.dy * Bi * Bj;
                    else
                        d = Bi * (Bj * (double)(-g.dz + g.rz + (R)zti * g.zz) * dztj + dBj * phi);
                } else if (b == 2) {
                    d = 2.0 * Bi * dBi * phi + Bi * Bi * 2.0 * (double)(g.rz + (R)zti * g.zz) * dzti;
                }
                acc[a] += d;
            }
        }
    }
    for (int a = 0; a < 3; ++a) red[a][l] = acc[a];
    __syncthreads();
    if (l < 3) {
        double t = 0.0;
        for (int k = 0; k < 64; ++k) t += red[l][k];
        div[3 * i + l] = mu0 * inv_a * t;
    }
}

}  // namespace

namespace {

// Symmetric VJP plan: groups of G blobs as for the product (64 only up to
// kSym64MaxN), 9 quantities per blob.
bool vjp_sym_plan(int64_t N, int prec, int ipw, int G, int* ng, int* C, int* Hmax, size_t* tb, size_t* sb) {
    if (G == 64 && N > kSym64MaxN) return false;
    *ng = (int)((N + G - 1) / G);
    *Hmax = *ng / 2;
    *C = (*Hmax + 1 + ipw - 1) / ipw;
    *tb = align_up((size_t)*ng * *C * kQ * G * sizeof(double));
    *sb = align_up((size_t)*ng * (*Hmax + 1) * kQ * G * real_size(prec));
    return *tb <= kSymPartialMaxBytes && *sb <= kSymPartialMaxBytes;
}

template <typename R, int NB>
void launch_vjp_sym(const R* rec, int ng, int C, int ipw, int Hmax, double* tpart, R* spart, hipStream_t st) {
    hipLaunchKernelGGL((sym_kernel<R, VjpBody<R>, NB>), dim3((unsigned)(ng * C)), dim3(64 * NB), 0, st, rec, ng, C,
                       ipw, Hmax, 1, tpart, spart, Box<R>{}, PackSrc{});
}

}  // namespace

size_t vjp_ws_bytes(int64_t N, int prec) {
    int splits;
    int64_t chunk;
    split_plan(N, 1, &splits, &chunk);
    size_t b = align_up((size_t)N * rec_width(prec, 2) * real_size(prec));
    b += align_up((size_t)N * sizeof(double));
    b += align_up((size_t)splits * kQ * N * sizeof(double));
    int ng, C, Hmax;
    size_t tb, sb;
    for (int G : {256, 64})
        if (vjp_sym_plan(N, prec, 1, G, &ng, &C, &Hmax, &tb, &sb)) {
            const size_t npad = (size_t)ng * G;
            const size_t s =
                align_up(npad * rec_width(prec, 2) * real_size(prec)) + align_up(npad * sizeof(double)) + tb + sb;
            b = std::max(b, s);
        }
    return b + 8 * kAlign;
}

int vjp(const double* pos, const double* f, const double* g, double* grad_pos, double* grad_f, int64_t N, double a,
        double eta, int prec, Arena& ar, hipStream_t st) {
    const size_t mark = ar.used;
    const int rw = rec_width(prec, 2);
    const Shape sh = tuned_shape(N, 1, prec);
    int ng, C, Hmax;
    size_t tb, sb;
    const int ipw = sh.ipw < 1 ? 1 : sh.ipw;
    int G = sym_group(sh.sym);
    bool sym = sh.sym && vjp_sym_plan(N, prec, ipw, G, &ng, &C, &Hmax, &tb, &sb);
    if (sh.sym && !sym && G == 64) {
        G = 256;
        sym = vjp_sym_plan(N, prec, ipw, G, &ng, &C, &Hmax, &tb, &sb);
    }
    const double m0 = 1.0 / (6.0 * M_PI * eta * a);
    const unsigned g1 = (unsigned)((N + kBlock - 1) / kBlock);
    if (sym) {
        const int64_t npad = (int64_t)ng * G;
        void* rec = ar.take((size_t)npad * rw * real_size(prec));
        double* B = (double*)ar.take((size_t)npad * sizeof(double));
        double* tpart = (double*)ar.take(tb);
        void* spart = ar.take(sb);
        if (!rec || !B || !tpart || !spart) {
            ar.used = mark;
            return RPYW_ENOMEM;
        }
        const unsigned gpk = (unsigned)((npad + kBlock - 1) / kBlock);  // records and padding
        hipEvent_t ev = nullptr;
        if (prec == RPYW_FP32C) {
            hipLaunchKernelGGL(pack_kernel<float>, dim3(gpk), dim3(kBlock), 0, st, pos, f, N, 2, rw, 1.0 / a,
                               (float*)rec, B, g, 0.0, 0.0, npad);
            RPYW_HIP(hipGetLastError());
            profile_begin(st, &ev);
            if (G == 64)
                launch_vjp_sym<float, 1>((const float*)rec, ng, C, ipw, Hmax, tpart, (float*)spart, st);
            else
                launch_vjp_sym<float, 4>((const float*)rec, ng, C, ipw, Hmax, tpart, (float*)spart, st);
            RPYW_HIP(hipGetLastError());
            profile_end(st, ev, (double)N * (double)N);
            hipLaunchKernelGGL(sym_vjp_epilogue<float>, dim3(g1), dim3(kBlock), 0, st, tpart, (const float*)spart, pos,
                               f, g, N, ng, C, Hmax, G, 1.0 / a, m0, grad_pos, grad_f);
        } else {
            hipLaunchKernelGGL(pack_kernel<double>, dim3(gpk), dim3(kBlock), 0, st, pos, f, N, 2, rw, 1.0 / a,
                               (double*)rec, B, g, 0.0, 0.0, npad);
            RPYW_HIP(hipGetLastError());
            profile_begin(st, &ev);
            if (G == 64)
                launch_vjp_sym<double, 1>((const double*)rec, ng, C, ipw, Hmax, tpart, (double*)spart, st);
            else
                launch_vjp_sym<double, 4>((const double*)rec, ng, C, ipw, Hmax, tpart, (double*)spart, st);
            RPYW_HIP(hipGetLastError());
            profile_end(st, ev, (double)N * (double)N);
            hipLaunchKernelGGL(sym_vjp_epilogue<double>, dim3(g1), dim3(kBlock), 0, st, tpart, (const double*)spart,
                               pos, f, g, N, ng, C, Hmax, G, 1.0 / a, m0, grad_pos, grad_f);
        }
        RPYW_HIP(hipGetLastError());
        ar.used = mark;
        return RPYW_OK;
    }
    void* rec = ar.take((size_t)N * rw * real_size(prec));
    double* B = (double*)ar.take((size_t)N * sizeof(double));
    int splits;
    int64_t chunk;
    split_plan(N, 1, &splits, &chunk);
    double* part = (double*)ar.take((size_t)splits * kQ * N * sizeof(double));
    if (!rec || !B || !part) {
        ar.used = mark;
        return RPYW_ENOMEM;
    }
    const int64_t nblocks = (int64_t)g1 * splits;
    hipEvent_t ev = nullptr;
    if (prec == RPYW_FP32C) {
        hipLaunchKernelGGL(pack_kernel<float>, dim3(g1), dim3(kBlock), 0, st, pos, f, N, 2, rw, 1.0 / a, (float*)rec, B,
                           g, 0.0, 0.0, N);
        RPYW_HIP(hipGetLastError());
        profile_begin(st, &ev);
        hipLaunchKernelGGL((vjp_kernel<float, 256>), dim3((unsigned)nblocks), dim3(kBlock), 0, st, (const float*)rec,
                           N, splits, chunk, part);
    } else {
        hipLaunchKernelGGL(pack_kernel<double>, dim3(g1), dim3(kBlock), 0, st, pos, f, N, 2, rw, 1.0 / a,
                           (double*)rec, B, g, 0.0, 0.0, N);
        RPYW_HIP(hipGetLastError());
        profile_begin(st, &ev);
        hipLaunchKernelGGL((vjp_kernel<double, 128>), dim3((unsigned)nblocks), dim3(kBlock), 0, st,
                           (const double*)rec, N, splits, chunk, part);
    }
    RPYW_HIP(hipGetLastError());
    profile_end(st, ev, (double)N * (double)N);
    hipLaunchKernelGGL(vjp_epilogue, dim3(g1), dim3(kBlock), 0, st, part, pos, f, g, N, splits, 1.0 / a, m0, grad_pos,
                       grad_f);
    RPYW_HIP(hipGetLastError());
    ar.used = mark;
    return RPYW_OK;
}

int divergence(const double* pos, double* div, int64_t N, double a, double eta, int prec, Arena&, hipStream_t st) {
    const unsigned g1 = (unsigned)N;  // one wave per target (N < 2^31)
    const double m0 = 1.0 / (6.0 * M_PI * eta * a);
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(divergence_kernel<float>, dim3(g1), dim3(64), 0, st, pos, N, 1.0 / a, m0, div);
    else
        hipLaunchKernelGGL(divergence_kernel<double>, dim3(g1), dim3(64), 0, st, pos, N, 1.0 / a, m0, div);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

}  // namespace rpyw
