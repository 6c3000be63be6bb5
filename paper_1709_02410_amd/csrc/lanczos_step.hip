// Fused steps of the preconditioned Lanczos iteration for M^{1/2} W
// (arXiv:1709.02410, Sec. II.B) when the product runs through the symmetric
// pair kernel.  Step k is four launches:
//   vin   one workgroup per body (per 21 blobs without bodies): the second
//         Gram-Schmidt correction and normalisation of the previous step,
//         v_k = (y' - V c2) / beta_{k-1}, with c2 = V^T y' and |y'|^2 added
//         up from the block partials of gs2 in a fixed order (every
//         workgroup repeats that small sum); then x = L^-T v_k, written
//         straight into the force slots of the pair kernel's records
//         (B x in the kernel precision; the positions are packed once);
//   pair  the symmetric pair kernel: M x as partial sums;
//   out   one workgroup per group of whole bodies (at most 64 entries, or
//         one larger body): y = M x gathered from the partial sums (eight
//         or four threads per entry, fixed order), w = L^-1 y -
//         beta_{k-1} v_{k-1} (the inverse factors staged through LDS), and
//         the group's partial dot products V_j . w (j <= k), one wave per
//         vector;
//   gs2   blocks of consecutive entries: c1 = V^T w added up from the
//         partials of out, alpha_k = c1[k], y' = w - V c1 (the first
//         correction), and the block partials of V^T y' and |y'|^2.
// The first correction and the second projection are the two classical
// Gram-Schmidt passes of the full reorthogonalisation; beta_k =
// (|y'|^2 - |c2|^2)^{1/2} as in the unfused driver.  vin of step k + 1 is
// launched with step k: its first workgroup publishes step k (alpha_k, kept
// in device memory by gs2, and beta_k into pinned memory, then, after a
// system-scope fence, the step's flag), so that the host sees both
// coefficients of a step when its flag is set.
#include <algorithm>
#include <cmath>
#include <vector>

#include "krylov_step.h"
#include "records.h"
#include "rpyw_internal.h"
#include "sym_pairs.h"

namespace rpyw {

namespace {

using namespace kstep;

constexpr int kVinThreads = 256;
constexpr int kOutThreads = 512;
constexpr int kGs2Threads = 256;
constexpr int kVinReg = 64;  // basis values vin keeps in registers
constexpr int kPackThreads = 256;

template <typename R>
__global__ __launch_bounds__(kVinThreads) void lz_vin_kernel(int diag, const int* __restrict__ units,
                                                             const int64_t* __restrict__ lofs,
                                                             const double* __restrict__ Lall, int64_t n3, int k,
                                                             const double* __restrict__ src,
                                                             const double* __restrict__ part2, int ncol2,
                                                             double* __restrict__ V, double* __restrict__ d_ab,
                                                             double* __restrict__ h_ab, double* __restrict__ h_flag,
                                                             R* __restrict__ rec, int recw,
                                                             const double* __restrict__ B,
                                                             double* __restrict__ h_hdr,
                                                             const int* __restrict__ bad0,
                                                             const int* __restrict__ bad1) {
    constexpr int PW = pos_slots<R>();
    __shared__ double c[kLanczosFusedMaxIter + 2];
    __shared__ double x[3 * kMaxBodyBlobs];
    __shared__ double Li[kLdsFactor];
    __shared__ double sinv;
    const int p = blockIdx.x, t = threadIdx.x;
    // The partials of gs2 first (they depend on nothing this kernel loads;
    // at k = 0 the packing kernel's partials of |W|^2): with up to 64 rows
    // of up to 64 columns, one batch of loads per lane (4 lanes per row),
    // added up after the other loads are issued.
    constexpr int kRl = 4;
    const bool one_batch = k + 1 <= kVinThreads / kRl && ncol2 <= kRl * kPre;
    const int rr = t / kRl, rq = t % kRl;
    double pv[kPre];
    if (one_batch && rr <= k) {
        const double* pr = part2 + (int64_t)rr * ncol2;
#pragma unroll
        for (int i = 0; i < kPre; ++i) pv[i] = pr[rq + kRl * i < ncol2 ? rq + kRl * i : ncol2 - 1];
    }
    const int64_t e0 = 3 * (int64_t)units[p];
    const int n = (int)(3 * (int64_t)units[p + 1] - e0);
    const bool lds_factor = !diag && n * n <= kLdsFactor;
    // loads that do not depend on the reductions go next: this entry's
    // source value, B of its blob, its basis values (the first kVinReg), and
    // the inverse factor
    Staged<kVinThreads, kLdsFactor / kVinThreads> sf;
    if (lds_factor) sf.load(Lall + 2 * lofs[p] + (int64_t)n * n, n * n);
    const int64_t e = e0 + t, ec = t < n ? e : e0;  // ec: an in-bounds address for idle lanes
    double vr = 0.0, bb = 0.0, a[kVinReg];
    if (t < n) {
        vr = src[e];
        bb = B[e / 3];
    }
#pragma unroll
    for (int j0 = 0; j0 < kVinReg; j0 += 16) {
        if (j0 >= k) break;  // uniform
#pragma unroll
        for (int j = j0; j < j0 + 16; ++j) a[j] = V[(j < k ? j : 0) * n3 + ec];
    }
    {
        // c[0..k) = c2, c[k] = |y'|^2 (k = 0: |W|^2); one pass over up to 64
        // rows
        if (one_batch) {
            double sr = 0.0;
#pragma unroll
            for (int i = 0; i < kPre; ++i)
                if (rq + kRl * i < ncol2) sr += pv[i];
            sr = lane_group_sum<kRl>(sr);
            if (rq == 0 && rr <= k) c[rr] = sr;
            __syncthreads();
        } else {
            reduce_rows<kVinThreads, 4, kPre>(part2, k + 1, ncol2, c);
        }
        if (t == 0) {
            double s2 = c[k];
            for (int j = 0; j < k; ++j) s2 -= c[j] * c[j];
            const double beta = s2 > 0.0 ? sqrt(s2) : 0.0;
            sinv = 1.0 / beta;  // beta = 0: breakdown, this step's values are discarded
            if (p == 0 && k > 0) {
                // publish step k - 1: alpha (kept by its gs2) and beta, then,
                // after a system-scope fence, its flag
                d_ab[2 * (k - 1) + 1] = beta;
                h_ab[2 * (k - 1)] = d_ab[2 * (k - 1)];
                h_ab[2 * (k - 1) + 1] = beta;
                __threadfence_system();
                h_flag[k - 1] = 1.0;
            } else if (p == 0) {
                // the call's header: beta_0 = |W| and the definiteness flags
                // of the factors; the host reads it with step 0, whose flag a
                // later kernel sets
                h_hdr[0] = beta;
                int* hb = reinterpret_cast<int*>(h_hdr + 1);
                hb[0] = bad0[0];
                hb[1] = bad1 ? bad1[0] : 0;
                __threadfence_system();
            }
        }
    }
    if (lds_factor) sf.store(Li, n * n);  // read after the next barrier
    __syncthreads();
    if (t < n) {
#pragma unroll
        for (int j = 0; j < kVinReg; ++j)
            if (j < k) vr -= c[j] * a[j];  // a[j] is V_j only for j < k
        for (int j0 = kVinReg; j0 < k; j0 += kPre) {
            double b[kPre];
#pragma unroll
            for (int j = 0; j < kPre; ++j) b[j] = j0 + j < k ? V[(j0 + j) * n3 + e] : 0.0;
#pragma unroll
            for (int j = 0; j < kPre; ++j)
                if (j0 + j < k) vr -= c[j0 + j] * b[j];
        }
        const double v = vr * sinv;
        V[k * n3 + e] = v;
        x[t] = v;
    }
    __syncthreads();
    if (t < n) {
        double s;
        if (diag) {
            s = x[t] / Lall[e];
        } else {
            // (L_p^-1)^T row t: column t of L_p^-1 from its diagonal down
            s = lds_factor ? dot4(Li + t * n + t, n, x + t, n - t)
                           : dot4(Lall + 2 * lofs[p] + (int64_t)n * n + t * n + t, n, x + t, n - t);
        }
        const int64_t blob = e / 3;
        rec[blob * recw + PW + (int)(e - 3 * blob)] = (R)(bb * s);
    }
}

template <typename R>
__global__ __launch_bounds__(kOutThreads) void lz_out_kernel(
    int diag, const int* __restrict__ units, const LanczosGroup* __restrict__ ginfo,
    const double* __restrict__ Lall, const double* __restrict__ tpart, const R* __restrict__ spart, int ng, int C,
    int Hmax, int nseg, int G, const double* __restrict__ B, double mu0, int64_t n3, int k,
    const double* __restrict__ V, const double* __restrict__ d_ab, double* __restrict__ w,
    double* __restrict__ part1, int ngroups, const double* __restrict__ ypre) {
    __shared__ double red[kOutThreads];
    __shared__ double y[3 * kMaxBodyBlobs];  // a group has at most 64 entries, or one body of up to 126
    __shared__ double wl[3 * kMaxBodyBlobs];
    __shared__ double Lf[2 * kLdsFactor];    // the group's factors as stored: L_p, then L_p^-1, per body
    __shared__ int ub[kLanczosGroupUnits + 1];
    const int g = blockIdx.x, t = threadIdx.x;
    // everything that does not depend on the product goes first: the group
    // (one table entry), then its unit offsets, factors, B, the previous
    // basis vector and beta_{k-1}, and the basis values of the dot products
    const LanczosGroup gi = ginfo[g];
    const int g0 = gi.g0, nu = gi.g1 - gi.g0;
    const int64_t e0 = 3 * (int64_t)gi.b0;
    const int n = 3 * (gi.b1 - gi.b0);
    // threads per entry: 8 for groups of up to 64 entries, 4 up to 128
    const int U = n <= 64 ? 8 : 4;
    const bool lds_factor = !diag && gi.sq <= kLdsFactor;
    const int uv = t <= nu ? units[g0 + t] : 0;
    Staged<kOutThreads, 2 * kLdsFactor / kOutThreads> sf;
    if (lds_factor) sf.load(Lall + 2 * gi.loff, 2 * gi.sq);
    double vprev = 0.0, bb = 0.0, dg = 0.0;
    if (t < n) {
        if (k > 0) vprev = V[(k - 1) * n3 + e0 + t];
        bb = B[(e0 + t) / 3];
        if (diag) dg = Lall[e0 + t];
    }
    const double bk = k > 0 ? d_ab[2 * (k - 1) + 1] : 0.0;
    // the lane's basis values for the dot products (waves take the vectors
    // j = wave (mod 8), lanes the entries l and l + 64), loaded ahead
    const int wv = t >> 6, l = t & 63;
    constexpr int kWaves = kOutThreads / 64;
    double av[kWaves][2];
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const int j = wv + kWaves * i;
        av[i][0] = (j <= k && l < n) ? V[j * n3 + e0 + l] : 0.0;
        av[i][1] = (j <= k && l + 64 < n) ? V[j * n3 + e0 + l + 64] : 0.0;
    }
    const int S = gather_slots(n);  // U = kOutThreads / S
    if (!ypre) {
        const int slot = t % S, u = t / S;
        double r = 0.0;
        if (slot < n) {
            const int64_t e = e0 + gather_entry(slot, n), blob = e / 3;
            r = gather_share<R>(tpart, spart, blob, ng, C, Hmax, nseg, G, (int)(e - 3 * blob), u, U);
        }
        red[t] = r;
    }
    if (t <= nu) ub[t] = uv;
    if (lds_factor) sf.store(Lf, 2 * gi.sq);
    __syncthreads();
    if (t < n && ypre) {
        y[t] = ypre[e0 + t];
    } else if (t < n) {
        const double* rt = red + gather_slot(t, n);
        double s = rt[0];
        if (U == 8) {
#pragma unroll
            for (int u = 1; u < 8; ++u) s += rt[u * 64];
        } else {
#pragma unroll
            for (int u = 1; u < 4; ++u) s += rt[u * 128];
        }
        y[t] = mu0 * bb * s;
    }
    __syncthreads();
    if (t < n) {
        const int64_t e = e0 + t;
        double v;
        if (diag) {
            v = y[t] / dg;
        } else {
            // the entry's body (unit offsets in LDS) and where its factors
            // start relative to the group's
            int q = 0, off = 0;
            while (3 * (ub[q + 1] - ub[0]) <= t) {
                const int nq = 3 * (ub[q + 1] - ub[q]);
                off += 2 * nq * nq;
                ++q;
            }
            const int bs = 3 * (ub[q] - ub[0]), bn = 3 * (ub[q + 1] - ub[q]);
            const int i = t - bs;
            const int64_t fi = off + (int64_t)bn * bn + (int64_t)i * bn;  // row i of L_p^-1
            v = lds_factor ? dot4(Lf + fi, 1, y + bs, i + 1) : dot4(Lall + 2 * gi.loff + fi, 1, y + bs, i + 1);
        }
        if (k > 0) v -= bk * vprev;
        w[e] = v;
        wl[t] = v;
    }
    __syncthreads();
    const double w0 = l < n ? wl[l] : 0.0, w1 = l + 64 < n ? wl[l + 64] : 0.0;
    {
        // the wave's kWaves dot products reduced together, one butterfly
        // level at a time (independent shuffles overlap)
        double pr[kWaves];
#pragma unroll
        for (int i = 0; i < kWaves; ++i) pr[i] = fma(av[i][1], w1, fma(av[i][0], w0, 0.0));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int i = 0; i < kWaves; ++i) pr[i] += __shfl_xor(pr[i], o, 64);
#pragma unroll
        for (int i = 0; i < kWaves; ++i) {
            const int j = wv + kWaves * i;
            if (l == 0 && j <= k) part1[(int64_t)j * ngroups + g] = pr[i];
        }
    }
    for (int j = wv + kWaves * kWaves; j <= k; j += kWaves) {
        const double* Vj = V + j * n3 + e0;
        double p = fma(l < n ? Vj[l] : 0.0, w0, 0.0);
        p = fma(l + 64 < n ? Vj[l + 64] : 0.0, w1, p);
        p = lane_group_sum<64>(p);
        if (l == 0) part1[(int64_t)j * ngroups + g] = p;
    }
}

// gs2: c1 from the partials of out; y' = w - sum_{j <= k} c1[j] V_j (terms
// subtracted in order); block partials of V_j . y' (j <= k) and |y'|^2.
// Block b takes kGs2Threads m consecutive entries, m per thread.  With one entry per
// thread and k < kGs2Reg, the entry's basis values are loaded once, before
// the reduction of c1, and serve both the update and the dot products.
constexpr int kGs2Reg = 64;
// Block 0 keeps the step's first projection for the next step's first
// kernel, which publishes the step: alpha_k = c1[k] into d_ab (Lanczos), or
// all of c1 into gc1 (GMRES).
__device__ __forceinline__ void keep_c1(int k, const double* c1, double* __restrict__ d_ab,
                                        double* __restrict__ gc1) {
    if (blockIdx.x != 0) return;
    if (gc1) {
        for (int j = threadIdx.x; j <= k; j += blockDim.x) gc1[j] = c1[j];
    } else if (threadIdx.x == 0) {
        d_ab[2 * k] = c1[k];
    }
}

__global__ __launch_bounds__(kGs2Threads) void lz_gs2_kernel(const double* __restrict__ w, double* __restrict__ yo,
                                                             int64_t n3, int m, const double* __restrict__ V, int k,
                                                             const double* __restrict__ part1, int ngroups,
                                                             double* __restrict__ part2, double* __restrict__ d_ab,
                                                             double* __restrict__ gc1) {
    constexpr int kBatch = 32;  // results per pass through the tile
    __shared__ double c1[kLanczosFusedMaxIter + 1];
    __shared__ double tile[kBatch][kGs2Threads + 1];
    const int t = threadIdx.x;
    const int nblk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * kGs2Threads * m + t;
    const int nd = k + 2;  // V_0 .. V_k, then |y'|^2
    // the tile's kBatch rows are added by kLpr lanes each
    constexpr int kLpr = kGs2Threads / kBatch;
    const int jr = t / kLpr, c0 = t % kLpr;
    if (m == 1 && k < kGs2Reg) {
        const bool has = base < n3;
        double a[kGs2Reg];
        double v = has ? w[base] : 0.0;
        const int64_t bc = has ? base : 0;  // an in-bounds address for idle lanes
#pragma unroll
        for (int j0 = 0; j0 < kGs2Reg; j0 += 16) {
            if (j0 > k) break;  // uniform
#pragma unroll
            for (int j = j0; j < j0 + 16; ++j) a[j] = V[(j <= k ? j : 0) * n3 + bc];
        }
        reduce_rows<kGs2Threads, 4, kPre>(part1, k + 1, ngroups, c1);  // one pass over up to 64 rows
        keep_c1(k, c1, d_ab, gc1);
#pragma unroll
        for (int j = 0; j < kGs2Reg; ++j)
            if (j <= k) v -= c1[j] * a[j];
        v = has ? v : 0.0;  // idle lanes: a[] holds values of entry 0, and they add nothing to the dots
        if (has) yo[base] = v;
        // batches of 16 results with compile-time indices into a[] (the
        // loops are fully unrolled; the last result is |y'|^2)
#pragma unroll
        for (int j0 = 0; j0 < kGs2Reg + kBatch; j0 += kBatch) {
            if (j0 >= nd) break;
            const int jn = nd - j0 < kBatch ? nd - j0 : kBatch;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int j = j0 + u;
                double p = 0.0;
                if (u < jn) {
                    if (j <= k) {
                        p = a[j < kGs2Reg ? j : 0] * v;
                    } else {
                        p = v * v;
                    }
                }
                tile[u][t] = p;
            }
            __syncthreads();
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < kGs2Threads / kLpr; ++i) s += tile[jr][c0 + kLpr * i];
            s = lane_group_sum<kLpr>(s);
            if (c0 == 0 && jr < jn) part2[(int64_t)(j0 + jr) * nblk + blockIdx.x] = s;
            __syncthreads();
        }
        return;
    }
    // general path: several entries per thread or many basis vectors
    reduce_rows<kGs2Threads>(part1, k + 1, ngroups, c1);
    keep_c1(k, c1, d_ab, gc1);
    double x[kLanczosGs2PerThread];
#pragma unroll
    for (int r = 0; r < kLanczosGs2PerThread; ++r) {
        const int64_t e = base + (int64_t)r * kGs2Threads;
        x[r] = 0.0;
        if (r >= m || e >= n3) continue;
        double v = w[e], a[kPre];
        for (int j0 = 0; j0 <= k; j0 += kPre) {
#pragma unroll
            for (int j = 0; j < kPre; ++j) a[j] = j0 + j <= k ? V[(j0 + j) * n3 + e] : 0.0;
#pragma unroll
            for (int j = 0; j < kPre; ++j)
                if (j0 + j <= k) v -= c1[j0 + j] * a[j];
        }
        yo[e] = v;
        x[r] = v;
    }
    for (int j0 = 0; j0 < nd; j0 += kBatch) {
        const int jn = nd - j0 < kBatch ? nd - j0 : kBatch;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            double p = 0.0;
            if (u < jn) {
                if (j0 + u <= k) {
                    const double* av = V + (j0 + u) * n3;
#pragma unroll
                    for (int r = 0; r < kLanczosGs2PerThread; ++r) {
                        const int64_t e = base + (int64_t)r * kGs2Threads;
                        if (r < m && e < n3) p = fma(av[e], x[r], p);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < kLanczosGs2PerThread; ++r) p = fma(x[r], x[r], p);
                }
            }
            tile[u][t] = p;
        }
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kGs2Threads / kLpr; ++i) s += tile[jr][c0 + kLpr * i];
        s = lane_group_sum<kLpr>(s);
        if (c0 == 0 && jr < jn) part2[(int64_t)(j0 + jr) * nblk + blockIdx.x] = s;
        __syncthreads();
    }
}

// The call's first kernel: the pair kernel's records of positions (and W
// in the force slots, which vin rewrites), B, and per block of 256 blobs
// the partial sum of |W_i|^2 (a fixed-order tree), from which vin of step 0
// forms beta_0 = |W|; block 0 also clears the definiteness flag that the
// factor build sets, which runs next.  The call's small tables (factor and
// gather offsets) come from pinned host memory with it, instead of a copy
// of their own.
template <typename R>
__global__ __launch_bounds__(kPackThreads) void lz_pack_kernel(const double* __restrict__ pos,
                                                               const double* __restrict__ W, int64_t N, int recw,
                                                               double inv_a, double lx, double ly, int64_t npad,
                                                               R* __restrict__ rec, double* __restrict__ B,
                                                               double* __restrict__ sqp, int* __restrict__ bad,
                                                               const int* __restrict__ htab, int* __restrict__ dtab,
                                                               int nwords) {
    __shared__ double red[kPackThreads];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kPackThreads + t;
    for (int64_t q = i; q < nwords; q += (int64_t)gridDim.x * kPackThreads) dtab[q] = htab[q];
    double w2 = 0.0;
    if (i < npad) {
        double b;
        make_record<R>(pos, W, N, 1, recw, inv_a, nullptr, lx, ly, i, rec + i * recw, &b);
        B[i] = b;
        if (i < N) w2 = W[3 * i] * W[3 * i] + W[3 * i + 1] * W[3 * i + 1] + W[3 * i + 2] * W[3 * i + 2];
    }
    red[t] = w2;
    __syncthreads();
    for (int h = kPackThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) {
        sqp[blockIdx.x] = red[0];
        if (blockIdx.x == 0) *bad = 0;
    }
}

// The call's last kernel: out = L (V c) per unit (body, or run of blobs),
// with the coefficients c passed by value.
struct LzCoefs {
    double c[kLanczosCoefArgs];
};
__global__ __launch_bounds__(kVinThreads) void lz_fin_kernel(int diag, const int* __restrict__ units,
                                                             const int64_t* __restrict__ lofs,
                                                             const double* __restrict__ Lall, int64_t n3,
                                                             const double* __restrict__ V, int nv, LzCoefs cf,
                                                             double* __restrict__ out) {
    __shared__ double y[3 * kMaxBodyBlobs];
    const int p = blockIdx.x, t = threadIdx.x;
    const int64_t e0 = 3 * (int64_t)units[p];
    const int n = (int)(3 * (int64_t)units[p + 1] - e0);
    double s = 0.0;
    if (t < n) {
        const double* v = V + e0 + t;
        double s1 = 0.0;
        int j = 0;
        for (; j + 1 < nv; j += 2) {
            s = fma(cf.c[j], v[j * n3], s);
            s1 = fma(cf.c[j + 1], v[(j + 1) * n3], s1);
        }
        if (j < nv) s = fma(cf.c[j], v[j * n3], s);
        s += s1;
        y[t] = s;
    }
    __syncthreads();
    if (t < n) {
        double o;
        if (diag) {
            o = Lall[e0 + t] * s;
        } else {
            const double* Lr = Lall + 2 * lofs[p] + (int64_t)t * n;  // row t of L_p
            o = 0.0;
            for (int m = 0; m <= t; ++m) o = fma(Lr[m], y[m], o);
        }
        out[e0 + t] = o;
    }
}

}  // namespace

bool lanczos_fused_applies(int64_t N, int prec, int max_iter, const Domain& dom, SymPlan* sp, int* ipw) {
    if (max_iter > kLanczosFusedMaxIter) return false;
    // the plan products() would use for one right-hand side
    const Shape sh = tuned_shape(N, 1, prec);
    if (!dom.periodic() && !(sh.sym && sh.kblk <= 4)) return false;
    const int w = sh.ipw < 1 ? 4 : sh.ipw;
    SymPlan p = sym_plan(N, prec, 1, w, dom.periodic() ? (sh.sym == 1 ? 256 : 64) : sym_group(sh.sym));
    if (!p.ok && p.G == 64) p = sym_plan(N, prec, 1, w, 256);
    if (!p.ok) return false;
    *sp = p;
    *ipw = w;
    return true;
}

int64_t lanczos_gs2_blocks(int64_t n3, int* m) {
    int mm = (int)((n3 + (int64_t)kGs2Threads * 1024 - 1) / ((int64_t)kGs2Threads * 1024));
    mm = std::max(1, std::min(mm, kLanczosGs2PerThread));
    *m = mm;
    return (n3 + (int64_t)kGs2Threads * mm - 1) / ((int64_t)kGs2Threads * mm);
}

// Units (blob offsets of the vin workgroups) and groups (unit offsets of the
// out workgroups: whole units of at most kLanczosOutEntries entries
// together, or one larger body alone) for bodies or, without bodies, for
// runs of kLanczosOutEntries / 3 blobs.
void lanczos_units(int64_t N, const int64_t* body_offsets, int n_bodies, std::vector<int>& units,
                   std::vector<int>& groups) {
    units.clear();
    groups.clear();
    if (n_bodies > 0) {
        for (int p = 0; p <= n_bodies; ++p) units.push_back((int)body_offsets[p]);
    } else {
        for (int64_t b = 0; b < N; b += kLanczosOutEntries / 3) units.push_back((int)b);
        units.push_back((int)N);
    }
    const int nu = (int)units.size() - 1;
    groups.push_back(0);
    int start = 0;
    for (int p = 0; p < nu; ++p) {
        if (p > start && 3 * (units[p + 1] - units[start]) > kLanczosOutEntries) {
            groups.push_back(p);
            start = p;
        }
    }
    groups.push_back(nu);
}

int lz_launch_vin(int prec, const BodyFactors& pc, const int* units, int nunits, int64_t n3, int k,
                  const double* src, const double* part2, int ncol2, double* V, double* d_ab, double* h_ab,
                  double* h_flag, void* rec, int recw, const double* B, double* h_hdr, const int* bad0,
                  const int* bad1, hipStream_t st) {
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(lz_vin_kernel<float>, dim3((unsigned)nunits), dim3(kVinThreads), 0, st, pc.diag ? 1 : 0,
                           units, pc.lofs, pc.L, n3, k, src, part2, ncol2, V, d_ab, h_ab, h_flag, (float*)rec, recw,
                           B, h_hdr, bad0, bad1);
    else
        hipLaunchKernelGGL(lz_vin_kernel<double>, dim3((unsigned)nunits), dim3(kVinThreads), 0, st, pc.diag ? 1 : 0,
                           units, pc.lofs, pc.L, n3, k, src, part2, ncol2, V, d_ab, h_ab, h_flag, (double*)rec, recw,
                           B, h_hdr, bad0, bad1);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int lz_launch_out(int prec, const BodyFactors& pc, const int* units, const LanczosGroup* ginfo, int ngroups,
                  const double* tpart, const void* spart, const SymPlan& sp, const double* B, double mu0, int64_t n3,
                  int k, const double* V, const double* d_ab, double* w, double* part1, const double* ypre,
                  hipStream_t st) {
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(lz_out_kernel<float>, dim3((unsigned)ngroups), dim3(kOutThreads), 0, st, pc.diag ? 1 : 0,
                           units, ginfo, pc.L, tpart, (const float*)spart, sp.ng, sp.C, sp.Hmax, sp.nseg, sp.G, B,
                           mu0, n3, k, V, d_ab, w, part1, ngroups, ypre);
    else
        hipLaunchKernelGGL(lz_out_kernel<double>, dim3((unsigned)ngroups), dim3(kOutThreads), 0, st, pc.diag ? 1 : 0,
                           units, ginfo, pc.L, tpart, (const double*)spart, sp.ng, sp.C, sp.Hmax, sp.nseg, sp.G, B,
                           mu0, n3, k, V, d_ab, w, part1, ngroups, ypre);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int64_t lz_pack_blocks(int64_t npad) { return (npad + kPackThreads - 1) / kPackThreads; }

int lz_launch_pack(int prec, const double* pos, const double* W, int64_t N, int64_t npad, int recw, double a,
                   const Domain& dom, void* rec, double* B, double* sqp, int* bad, const int* htab, int* dtab,
                   int nwords, hipStream_t st) {
    const unsigned g = (unsigned)lz_pack_blocks(npad);
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(lz_pack_kernel<float>, dim3(g), dim3(kPackThreads), 0, st, pos, W, N, recw, 1.0 / a,
                           dom.lx / a, dom.ly / a, npad, (float*)rec, B, sqp, bad, htab, dtab, nwords);
    else
        hipLaunchKernelGGL(lz_pack_kernel<double>, dim3(g), dim3(kPackThreads), 0, st, pos, W, N, recw, 1.0 / a,
                           dom.lx / a, dom.ly / a, npad, (double*)rec, B, sqp, bad, htab, dtab, nwords);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int lz_launch_fin(const BodyFactors& pc, const int* units, int nunits, int64_t n3, const double* V, const double* c,
                  int nv, double* out, hipStream_t st) {
    if (nv < 1 || nv > kLanczosCoefArgs) return RPYW_EINVAL;
    LzCoefs cf;
    for (int j = 0; j < kLanczosCoefArgs; ++j) cf.c[j] = j < nv ? c[j] : 0.0;
    hipLaunchKernelGGL(lz_fin_kernel, dim3((unsigned)nunits), dim3(kVinThreads), 0, st, pc.diag ? 1 : 0, units,
                       pc.lofs, pc.L, n3, V, nv, cf, out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int lz_launch_gs2(const double* w, double* yo, int64_t n3, const double* V, int k, const double* part1, int ngroups,
                  double* part2, double* d_ab, double* gc1, hipStream_t st) {
    int m;
    const int64_t nb = lanczos_gs2_blocks(n3, &m);
    hipLaunchKernelGGL(lz_gs2_kernel, dim3((unsigned)nb), dim3(kGs2Threads), 0, st, w, yo, n3, m, V, k, part1, ngroups,
                       part2, d_ab, gc1);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

}  // namespace rpyw
