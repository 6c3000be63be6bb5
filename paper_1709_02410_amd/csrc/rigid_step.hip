// Fused Arnoldi steps of the preconditioned GMRES solve of the rigid
// multiblob system (arXiv:1709.02410, Sec. II.A for the system, Sec. II.B
// for the block-diagonal preconditioner) when the product by M runs
// through the symmetric pair kernel.  Step k is four launches:
//   pre   one workgroup per body: c2 = V^T y' and |y'|^2 of step k - 1
//         added up from the block partials of its gs2 in a fixed order
//         (every workgroup repeats that small sum), h = (|y'|^2 -
//         |c2|^2)^{1/2}, and v_k = (y' - V c2) / h, the second Gram-Schmidt
//         correction (b / |b| at k = 0, |b|^2 from the block partials of
//         the right-hand side kernel), stored as basis vector k;
//         z = P^-1 v_k for the body (the exact inverse of its own
//         saddle-point block, factors staged through LDS); B z_lambda
//         written straight into the force slots of the pair kernel's
//         records (the positions are packed once);
//   pair  the symmetric pair kernel: M z_lambda as partial sums;
//   out   one workgroup per body: y = M z_lambda gathered from the partial
//         sums in a fixed order, w = A z = [y - K z_U | -K^T z_lambda], and
//         the body's partial dot products V_j . w (j <= k);
//   gs2   the Lanczos gs2 kernel: c1 = V^T w (kept for the next pre),
//         y' = w - V c1, and the block partials of V^T y' and |y'|^2.
// The pre kernel of step k + 1 is launched with step k: its first
// workgroup publishes the Hessenberg column of step k ([c1, c2, h] into a
// pinned slot, then, after a system-scope fence, the step's flag).
#include <algorithm>
#include <cmath>
#include <vector>

#include "krylov_step.h"
#include "records.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

using namespace kstep;

constexpr int kPreThreads = 256;  // at least 3 kMaxBodyBlobs + 6 (one thread per entry)
constexpr int kOutThreads = 256;
constexpr int kMaxN3 = 3 * kMaxBodyBlobs;
constexpr int kPreReg = 64;  // basis values pre keeps in registers
constexpr int kRhsThreads = 256;

template <typename R>
__global__ __launch_bounds__(kPreThreads) void rg_pre_kernel(
    const double* __restrict__ Lall, const int* __restrict__ bofs, const int64_t* __restrict__ lofs,
    const double* __restrict__ Wall, const double* __restrict__ Nall, int64_t n3, int64_t ld,
    const double* __restrict__ src, const double* __restrict__ part2, int ncol2, const double* __restrict__ gc1,
    double* __restrict__ hslots, int slot, double* __restrict__ h_flag, int k, double* __restrict__ V,
    double* __restrict__ zl, double* __restrict__ zu, R* __restrict__ rec, int recw, const double* __restrict__ B,
    double* __restrict__ h_hdr, const int* __restrict__ bad0, const int* __restrict__ bad1) {
    constexpr int PW = pos_slots<R>();
    __shared__ double cs[kLanczosFusedMaxIter + 1];
    __shared__ double r[kMaxN3 + 6], t1[kMaxN3], tt[kMaxN3];
    __shared__ double Ls[kLdsFactor];
    __shared__ double Ws[6 * kMaxN3];
    __shared__ double s6[6], z6[6], sc;
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = bofs[p], n = 3 * (bofs[p + 1] - b0);
    const int64_t e0 = 3 * (int64_t)b0;
    const bool lds_factor = n * n <= kLdsFactor;
    const double* Li = Lall + 2 * lofs[p] + (int64_t)n * n;
    const double* W = Wall + 18 * (int64_t)b0;
    // everything the step does not compute goes first: the factors, the
    // input entry and its basis values, N_p, c2 and the scale
    Staged<kPreThreads, kLdsFactor / kPreThreads> sl;
    if (lds_factor) sl.load(Li, n * n);
    Staged<kPreThreads, (6 * kMaxN3 + kPreThreads - 1) / kPreThreads> sw;
    sw.load(W, 6 * n);
    // thread t < n: lambda entry t; n <= t < n + 6: U entry t - n
    const bool has = t < n + 6;
    const int64_t e = t < n ? e0 + t : n3 + 6 * (int64_t)p + (t - n);
    const int64_t ec = has ? e : e0;  // an in-bounds address for idle lanes
    double x = has ? src[e] : 0.0, a[kPreReg];
#pragma unroll
    for (int j0 = 0; j0 < kPreReg; j0 += 16) {
        if (j0 >= k) break;  // uniform
#pragma unroll
        for (int j = j0; j < j0 + 16; ++j) a[j] = V[(j < k ? j : 0) * ld + ec];
    }
    double np[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (t < 6)
#pragma unroll
        for (int c = 0; c < 6; ++c) np[c] = Nall[36 * (int64_t)p + 6 * t + c];
    // c2 of step k - 1 into cs[0..k), |y'|^2 into cs[k] (k = 0: |b|^2 from
    // the right-hand side kernel's partials)
    reduce_rows<kPreThreads, 4, kPre>(part2, k + 1, ncol2, cs);
    if (t == 0) {
        double s2 = cs[k];
        for (int j = 0; j < k; ++j) s2 -= cs[j] * cs[j];
        const double h = s2 > 0.0 ? sqrt(s2) : 0.0;
        sc = h;  // h = 0: breakdown, this step's values are discarded
        if (p == 0 && k > 0) {
            hslots[(size_t)((k - 1) % PinnedSlots::kSlots) * slot + 2 * k] = h;
        } else if (p == 0) {
            // the call's header: |b| and the definiteness flags of the
            // factors; the host reads it with step 0, whose flag a later
            // kernel sets
            h_hdr[0] = h;
            int* hb = reinterpret_cast<int*>(h_hdr + 1);
            hb[0] = bad0[0];
            hb[1] = bad1 ? bad1[0] : 0;
            __threadfence_system();
        }
    }
    if (k > 0) {
        if (p == 0) {
            // publish column k - 1: c1 (kept by its gs2), c2, h; then its flag
            double* hc = hslots + (size_t)((k - 1) % PinnedSlots::kSlots) * slot;
            for (int j = t; j < k; j += kPreThreads) {
                hc[j] = gc1[j];
                hc[k + j] = cs[j];
            }
            __threadfence_system();
            __syncthreads();
            if (t == 0) h_flag[k - 1] = 1.0;
        }
    }
    if (lds_factor) sl.store(Ls, n * n);
    sw.store(Ws, 6 * n);
    __syncthreads();
    if (has) {
#pragma unroll
        for (int j = 0; j < kPreReg; ++j)
            if (j < k) x -= cs[j] * a[j];  // a[j] is V_j only for j < k
        for (int j0 = kPreReg; j0 < k; j0 += kPre) {
            double b[kPre];
#pragma unroll
            for (int j = 0; j < kPre; ++j) b[j] = j0 + j < k ? V[(j0 + j) * ld + e] : 0.0;
#pragma unroll
            for (int j = 0; j < kPre; ++j)
                if (j0 + j < k) x -= cs[j0 + j] * b[j];
        }
        const double v = x / sc;
        V[(int64_t)k * ld + e] = v;
        r[t] = v;  // lambda entries, then the six U entries at r[n ..]
    }
    __syncthreads();
    // t1 = L^-1 r_lambda; s = W^T r_lambda (six sums of 16 lanes each)
    if (t < n) t1[t] = lds_factor ? dot4(Ls + t * n, 1, r, t + 1) : dot4(Li + (int64_t)t * n, 1, r, t + 1);
    if (t < 96) {
        const int c = t >> 4, l16 = t & 15;
        double s = 0.0;
        for (int i = l16; i < n; i += 16) s = fma(Ws[6 * i + c], r[i], s);
        s = lane_group_sum<16>(s);
        if (l16 == 0) s6[c] = s;
    }
    __syncthreads();
    // tt = L^-T t1 = M_pp^-1 r_lambda; z_U = -N_p (r_U + s)
    if (t < n)
        tt[t] = lds_factor ? dot4(Ls + t * n + t, n, t1 + t, n - t)
                           : dot4(Li + (int64_t)t * n + t, n, t1 + t, n - t);
    if (t < 6) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) s = fma(np[c], r[n + c] + s6[c], s);
        z6[t] = -s;
        zu[6 * (int64_t)p + t] = -s;
    }
    __syncthreads();
    // z_lambda = tt + W z_U, and the records' force slots B z_lambda
    if (t < n) {
        double s = tt[t];
#pragma unroll
        for (int c = 0; c < 6; ++c) s = fma(Ws[6 * t + c], z6[c], s);
        zl[e0 + t] = s;
        const int64_t blob = (e0 + t) / 3;
        rec[blob * recw + PW + (int)(e0 + t - 3 * blob)] = (R)(B[blob] * s);
    }
}

// The call's first kernel: the right-hand side b = [-slip | -F, -T] of the
// saddle-point system, per block the partial sum of |b_e|^2 (a fixed-order
// tree; pre of step 0 forms |b| from them), the pair kernel's records of
// the positions with zero force slots (pre rewrites those every step) and
// B, the call's tables from pinned host memory (htab, nwords ints), and
// block 0 clears the definiteness flag that the factor kernels, which run
// next, set.
template <typename R>
__global__ __launch_bounds__(kRhsThreads) void rg_rhs_kernel(const double* __restrict__ pos, int64_t N, int64_t npad,
                                                             int recw, double inv_a, double lx, double ly,
                                                             R* __restrict__ rec, double* __restrict__ B,
                                                             const double* __restrict__ slip,
                                                             const double* __restrict__ FT, int64_t n3, int64_t n6,
                                                             double* __restrict__ b, double* __restrict__ sqp,
                                                             int* __restrict__ bad, const int* __restrict__ htab,
                                                             int* __restrict__ dtab, int nwords) {
    __shared__ double red[kRhsThreads];
    const int t = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x * kRhsThreads + t, stride = (int64_t)gridDim.x * kRhsThreads;
    for (int64_t q = e; q < nwords; q += stride) dtab[q] = htab[q];
    for (int64_t i = e; i < npad; i += stride) {
        double bb;
        make_record<R>(pos, nullptr, N, 0, recw, inv_a, nullptr, lx, ly, i, rec + i * recw, &bb);
        B[i] = bb;
    }
    double v = 0.0;
    if (e < n3)
        v = slip ? -slip[e] : 0.0;
    else if (e < n3 + n6)
        v = FT ? -FT[e - n3] : 0.0;
    if (e < n3 + n6) b[e] = v;
    red[t] = v * v;
    __syncthreads();
    for (int h = kRhsThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) {
        sqp[blockIdx.x] = red[0];
        if (blockIdx.x == 0) *bad = 0;
    }
}

// The solve's last kernel: x = P^-1 (V y) per body, the coefficients y
// passed by value: r = sum_j y_j V_j over the body's lambda entries and its
// six U entries, then the body's exact saddle-point inverse as in pre
// (M_pp^-1 = L^-T L^-1, z_U = -N_p (r_U + W^T r_lambda), z_lambda =
// M_pp^-1 r_lambda + W z_U), into the caller's outputs.
struct RgCoefs {
    double y[kLanczosCoefArgs];
};
__global__ __launch_bounds__(kPreThreads) void rg_fin_kernel(const double* __restrict__ Lall,
                                                             const int* __restrict__ bofs,
                                                             const int64_t* __restrict__ lofs,
                                                             const double* __restrict__ Wall,
                                                             const double* __restrict__ Nall, int64_t n3, int64_t ld,
                                                             const double* __restrict__ V, int nv, RgCoefs cf,
                                                             double* __restrict__ lam_out,
                                                             double* __restrict__ U_out) {
    __shared__ double r[kMaxN3 + 6], t1[kMaxN3], tt[kMaxN3];
    __shared__ double s6[6], z6[6];
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = bofs[p], n = 3 * (bofs[p + 1] - b0);
    const int64_t e0 = 3 * (int64_t)b0;
    const double* Li = Lall + 2 * lofs[p] + (int64_t)n * n;
    const double* W = Wall + 18 * (int64_t)b0;
    if (t < n + 6) {
        const int64_t e = t < n ? e0 + t : n3 + 6 * (int64_t)p + (t - n);
        const double* v = V + e;
        double s0 = 0.0, s1 = 0.0;
        int j = 0;
        for (; j + 1 < nv; j += 2) {
            s0 = fma(cf.y[j], v[j * ld], s0);
            s1 = fma(cf.y[j + 1], v[(j + 1) * ld], s1);
        }
        if (j < nv) s0 = fma(cf.y[j], v[j * ld], s0);
        r[t] = s0 + s1;
    }
    __syncthreads();
    if (t < n) t1[t] = dot4(Li + (int64_t)t * n, 1, r, t + 1);  // row t of L^-1
    if (t < 96) {
        const int c = t >> 4, l16 = t & 15;
        double s = 0.0;
        for (int i = l16; i < n; i += 16) s = fma(W[6 * i + c], r[i], s);
        s = lane_group_sum<16>(s);
        if (l16 == 0) s6[c] = s;
    }
    __syncthreads();
    if (t < n) tt[t] = dot4(Li + (int64_t)t * n + t, n, t1 + t, n - t);  // row t of L^-T
    if (t < 6) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) s = fma(Nall[36 * (int64_t)p + 6 * t + c], r[n + c] + s6[c], s);
        z6[t] = -s;
        U_out[6 * (int64_t)p + t] = -s;
    }
    __syncthreads();
    if (t < n) {
        double s = tt[t];
#pragma unroll
        for (int c = 0; c < 6; ++c) s = fma(W[6 * t + c], z6[c], s);
        lam_out[e0 + t] = s;
    }
}

template <typename R>
__global__ __launch_bounds__(kOutThreads) void rg_out_kernel(
    const double* __restrict__ pos, const double* __restrict__ q, const int* __restrict__ bofs,
    const double* __restrict__ tpart, const R* __restrict__ spart, int ng, int C, int Hmax, int nseg, int G,
    const double* __restrict__ B, double mu0, const double* __restrict__ zl, const double* __restrict__ zu,
    int64_t n3, int64_t ld, const double* __restrict__ V, int k, double* __restrict__ w,
    double* __restrict__ part1, int nbodies, const double* __restrict__ ypre) {
    constexpr int kWaves = kOutThreads / 64;
    constexpr int kSlots = 3;  // entries per lane for the dot products (n + 6 <= 132)
    __shared__ double red[kOutThreads];
    __shared__ double wl[kMaxN3 + 6];
    __shared__ double ur[6][kMaxBodyBlobs];
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = bofs[p], nb = bofs[p + 1] - b0, n = 3 * nb, ne = n + 6;
    const int64_t e0 = 3 * (int64_t)b0;
    // loads that do not depend on the product first
    double zu6[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) zu6[c] = zu[6 * (int64_t)p + c];
    double d[3] = {0.0, 0.0, 0.0}, bb = 0.0;
    if (t < n) {
        const int64_t blob = b0 + t / 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = pos[3 * blob + c] - q[3 * (int64_t)p + c];
        bb = B[blob];
    }
    double lam[3] = {0.0, 0.0, 0.0}, db[3] = {0.0, 0.0, 0.0};
    if (t < nb) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lam[c] = zl[e0 + 3 * t + c];
            db[c] = pos[3 * (b0 + t) + c] - q[3 * (int64_t)p + c];
        }
    }
    // the lane's basis values for the dot products: waves take the vectors
    // j = wave (mod kWaves), lanes the entries l, l + 64, l + 128
    const int wv = t >> 6, l = t & 63;
    auto gidx = [&](int i) -> int64_t { return i < n ? e0 + i : n3 + 6 * (int64_t)p + (i - n); };
    constexpr int kJ = 64 / kWaves;  // vectors per wave held in registers (j < 64)
    double av[kJ][kSlots];
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        const int j = wv + kWaves * i;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int idx = l + 64 * s;
            av[i][s] = (j <= k && idx < ne) ? V[(int64_t)j * ld + gidx(idx)] : 0.0;
        }
    }
    // y = M z_lambda: U threads per entry add their share of the partials
    const int U = n <= 64 ? 4 : 2;
    const int S = gather_slots(n);  // U = kOutThreads / S
    if (!ypre) {
        const int slot = t % S, u = t / S;
        double rr = 0.0;
        if (slot < n) {
            const int64_t e = e0 + gather_entry(slot, n), blob = e / 3;
            rr = gather_share<R>(tpart, spart, blob, ng, C, Hmax, nseg, G, (int)(e - 3 * blob), u, U);
        }
        red[t] = rr;
    }
    // -K^T z_lambda: per blob the force and its torque about q
    if (t < nb) {
        ur[0][t] = lam[0];
        ur[1][t] = lam[1];
        ur[2][t] = lam[2];
        ur[3][t] = db[1] * lam[2] - db[2] * lam[1];
        ur[4][t] = db[2] * lam[0] - db[0] * lam[2];
        ur[5][t] = db[0] * lam[1] - db[1] * lam[0];
    }
    __syncthreads();
    if (t < n) {
        double y;
        if (ypre) {
            y = ypre[e0 + t];
        } else {
            const int slot = gather_slot(t, n);
            double s = red[slot];
            for (int u = 1; u < U; ++u) s += red[u * S + slot];
            y = mu0 * bb * s;
        }
        // (K z_U) for this entry's component: u + omega x d
        const int al = t % 3;
        const double ku = al == 0   ? zu6[0] + zu6[4] * d[2] - zu6[5] * d[1]
                          : al == 1 ? zu6[1] + zu6[5] * d[0] - zu6[3] * d[2]
                                    : zu6[2] + zu6[3] * d[1] - zu6[4] * d[0];
        const double v = y - ku;
        w[e0 + t] = v;
        wl[t] = v;
    } else if (t >= 64 * (kWaves - 1) && t - 64 * (kWaves - 1) < 6) {
        // the last wave's first six lanes (idle in the gather for n < 192)
        const int c = t - 64 * (kWaves - 1);
        double s = 0.0;
        for (int a = 0; a < nb; ++a) s += ur[c][a];
        w[n3 + 6 * (int64_t)p + c] = -s;
        wl[n + c] = -s;
    }
    __syncthreads();
    double wv3[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) wv3[s] = l + 64 * s < ne ? wl[l + 64 * s] : 0.0;
    double pr[kJ];
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kSlots; ++c) s = fma(av[i][c], wv3[c], s);
        pr[i] = s;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < kJ; ++i) pr[i] += __shfl_xor(pr[i], o, 64);
#pragma unroll
    for (int i = 0; i < kJ; ++i) {
        const int j = wv + kWaves * i;
        if (l == 0 && j <= k) part1[(int64_t)j * nbodies + p] = pr[i];
    }
    for (int j = wv + 64; j <= k; j += kWaves) {  // beyond the vectors held in registers
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kSlots; ++c) {
            const int idx = l + 64 * c;
            if (idx < ne) s = fma(V[(int64_t)j * ld + gidx(idx)], wv3[c], s);
        }
        s = lane_group_sum<64>(s);
        if (l == 0) part1[(int64_t)j * nbodies + p] = s;
    }
}

}  // namespace

int rg_launch_pre(int prec, const BodyFactors& pc, const double* Wall, const double* Nall, int n_bodies, int64_t n3,
                  int64_t ld, const double* src, const double* part2, int ncol2, const double* gc1, double* hslots,
                  int slot, double* h_flag, int k, double* V, double* zl, double* zu, void* rec, int recw,
                  const double* B, double* h_hdr, const int* bad0, const int* bad1, hipStream_t st) {
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(rg_pre_kernel<float>, dim3((unsigned)n_bodies), dim3(kPreThreads), 0, st, pc.L, pc.bofs,
                           pc.lofs, Wall, Nall, n3, ld, src, part2, ncol2, gc1, hslots, slot, h_flag, k, V, zl, zu,
                           (float*)rec, recw, B, h_hdr, bad0, bad1);
    else
        hipLaunchKernelGGL(rg_pre_kernel<double>, dim3((unsigned)n_bodies), dim3(kPreThreads), 0, st, pc.L, pc.bofs,
                           pc.lofs, Wall, Nall, n3, ld, src, part2, ncol2, gc1, hslots, slot, h_flag, k, V, zl, zu,
                           (double*)rec, recw, B, h_hdr, bad0, bad1);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int rg_launch_fin(const BodyFactors& pc, const double* Wall, const double* Nall, int n_bodies, int64_t n3, int64_t ld,
                  const double* V, const double* y, int nv, double* lam_out, double* U_out, hipStream_t st) {
    if (nv < 1 || nv > kLanczosCoefArgs) return RPYW_EINVAL;
    RgCoefs cf;
    for (int j = 0; j < kLanczosCoefArgs; ++j) cf.y[j] = j < nv ? y[j] : 0.0;
    hipLaunchKernelGGL(rg_fin_kernel, dim3((unsigned)n_bodies), dim3(kPreThreads), 0, st, pc.L, pc.bofs, pc.lofs, Wall,
                       Nall, n3, ld, V, nv, cf, lam_out, U_out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int64_t rg_rhs_blocks(int64_t n) { return (n + kRhsThreads - 1) / kRhsThreads; }

int rg_launch_rhs(int prec, const double* pos, int64_t N, int64_t npad, int recw, double a, const Domain& dom,
                  void* rec, double* B, const double* slip, const double* FT, int64_t n3, int64_t n6, double* b,
                  double* sqp, int* bad, const int* htab, int* dtab, int nwords, hipStream_t st) {
    const unsigned g = (unsigned)rg_rhs_blocks(n3 + n6);
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(rg_rhs_kernel<float>, dim3(g), dim3(kRhsThreads), 0, st, pos, N, npad, recw, 1.0 / a,
                           dom.lx / a, dom.ly / a, (float*)rec, B, slip, FT, n3, n6, b, sqp, bad, htab, dtab, nwords);
    else
        hipLaunchKernelGGL(rg_rhs_kernel<double>, dim3(g), dim3(kRhsThreads), 0, st, pos, N, npad, recw, 1.0 / a,
                           dom.lx / a, dom.ly / a, (double*)rec, B, slip, FT, n3, n6, b, sqp, bad, htab, dtab,
                           nwords);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int rg_launch_out(int prec, const double* pos, const double* q, const int* bofs, int n_bodies, const double* tpart,
                  const void* spart, const SymPlan& sp, const double* B, double mu0, const double* zl,
                  const double* zu, int64_t n3, int64_t ld, const double* V, int k, double* w, double* part1,
                  const double* ypre, hipStream_t st) {
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(rg_out_kernel<float>, dim3((unsigned)n_bodies), dim3(kOutThreads), 0, st, pos, q, bofs,
                           tpart, (const float*)spart, sp.ng, sp.C, sp.Hmax, sp.nseg, sp.G, B, mu0, zl, zu, n3, ld, V,
                           k, w, part1, n_bodies, ypre);
    else
        hipLaunchKernelGGL(rg_out_kernel<double>, dim3((unsigned)n_bodies), dim3(kOutThreads), 0, st, pos, q, bofs,
                           tpart, (const double*)spart, sp.ng, sp.C, sp.Hmax, sp.nseg, sp.G, B, mu0, zl, zu, n3, ld,
                           V, k, w, part1, n_bodies, ypre);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

}  // namespace rpyw
