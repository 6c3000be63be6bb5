// Dense O(N^2) products u = M(r) f of the wall-corrected RPY blob mobility
// (arXiv:1709.02410, Sec. II.A: direct summation over all blob pairs, the
// operation whose cost dominates every Brownian-dynamics step).
//
// Pipeline per pass of kb right-hand sides:
//   pack      O(N):   AoS FP64 [N][3] -> one record per blob in the kernel
//                     precision: scaled position (x, y, z~) (+ FP32 low parts
//                     of x and y), then B_j f_j for each RHS.
//   pair      O(N^2): workgroup = 256*TPL targets x one source chunk; source
//                     records are staged through LDS tiles, every lane keeps
//                     its targets' sums in registers.  FP32 sums are plain
//                     within a tile and folded into a TwoSum (hi, lo) pair
//                     after each tile.  Partial sums per source chunk go to
//                     the workspace.
//   epilogue  O(N):   fixed-order sum of the chunk partials, times
//                     mu0 * B_i, written as FP64 [N][3].
// No floating-point atomics: results are bitwise reproducible for a fixed
// launch shape.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "pair_math.h"
#include "records.h"
#include "rpyw_internal.h"
#include "mat_pairs.h"
#include "sym_pairs.h"

namespace rpyw {

namespace {

// Targets held by one lane.
template <typename R, int K, int TPL>
struct Lane {
    R x[TPL], y[TPL], z[TPL], xl[TPL], yl[TPL];
    R acc[TPL][K][3];
    R hi[TPL][K][3], lo[TPL][K][3];  // FP32 compensated running sums

    __device__ void load(const R* __restrict__ rec, int64_t first, int64_t last, int64_t tid) {
        constexpr int RW = rec_w<R, K>();
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            int64_t i = first + (int64_t)t * kBlock + tid;
            if (i >= last) i = last - 1;
            const R* r = rec + i * RW;
            x[t] = r[0];
            y[t] = r[1];
            z[t] = r[2];
            if constexpr (sizeof(R) == 4) {
                xl[t] = r[3];
                yl[t] = r[4];
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    acc[t][k][c] = R(0);
                    hi[t][k][c] = R(0);
                    lo[t][k][c] = R(0);
                }
        }
    }

    // Sum over sources [s0, s1) staged through the LDS tile.
    template <int TILE>
    __device__ void run(const R* __restrict__ rec, int64_t s0, int64_t s1, R* tile) {
        constexpr int RW = rec_w<R, K>();
        constexpr int PW = pos_slots<R>();
        for (int64_t t0 = s0; t0 < s1; t0 += TILE) {
            const int n = (int)((s1 - t0) < TILE ? (s1 - t0) : TILE);
            __syncthreads();
            const R* g = rec + t0 * RW;
            for (int e = threadIdx.x; e < n * RW; e += kBlock) tile[e] = g[e];
            __syncthreads();
#pragma unroll 2
            for (int j = 0; j < n; ++j) {
                const R* s = tile + j * RW;
                const R sx = s[0], sy = s[1], sz = s[2];
                R sxl = R(0), syl = R(0);
                if constexpr (sizeof(R) == 4) {
                    sxl = s[3];
                    syl = s[4];
                }
#pragma unroll
                for (int t = 0; t < TPL; ++t) {
                    R dx = x[t] - sx, dy = y[t] - sy;
                    if constexpr (sizeof(R) == 4) {
                        dx += xl[t] - sxl;
                        dy += yl[t] - syl;
                    }
                    const R dz = z[t] - sz;
                    const PairCoef<R> p = pair_coef<R>(dx, dy, dz, z[t], sz);
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        pair_apply<R>(p, dx, dy, dz, s[PW + 3 * k], s[PW + 3 * k + 1], s[PW + 3 * k + 2],
                                      acc[t][k][0], acc[t][k][1], acc[t][k][2]);
                }
            }
            if constexpr (sizeof(R) == 4) {
#pragma unroll
                for (int t = 0; t < TPL; ++t)
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            two_sum_acc(hi[t][k][c], lo[t][k][c], acc[t][k][c]);
                            acc[t][k][c] = R(0);
                        }
            }
        }
    }

    __device__ double total(int t, int k, int c) const {
        if constexpr (sizeof(R) == 4)
            return (double)hi[t][k][c] + (double)lo[t][k][c];
        else
            return (double)acc[t][k][c];
    }
};

// Plain product: block b -> (source chunk b % splits, target block b / splits).
// With splits a multiple of 8, all workgroups of one XCD (dispatched
// round-robin by block index) read the same source chunk.
template <typename R, int K, int TPL, int TILE>
__global__ __launch_bounds__(kBlock) void pair_kernel(const R* __restrict__ rec, int64_t N, int splits,
                                                      int64_t chunk, double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) R tile[TILE * rec_w<R, K>()];
    const int b = blockIdx.x;
    const int split = b % splits;
    const int64_t first = (int64_t)(b / splits) * kBlock * TPL;
    const int64_t s0 = (int64_t)split * chunk;
    const int64_t s1 = s0 + chunk < N ? s0 + chunk : N;
    Lane<R, K, TPL> L;
    L.load(rec, first, N, threadIdx.x);
    L.template run<TILE>(rec, s0, s1, tile);
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
        const int64_t i = first + (int64_t)t * kBlock + threadIdx.x;
        if (i >= N) continue;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) part[((int64_t)(split * K + k) * 3 + c) * N + i] = L.total(t, k, c);
    }
}

// U[k][i][c] = mu0 B_i sum_s part[s][k][c][i] for k < kb (fixed order in s).
__global__ void epilogue_kernel(const double* __restrict__ part, const double* __restrict__ B, int64_t N, int kdim,
                                int kb, int splits, double mu0, double* __restrict__ U) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double sc = mu0 * B[i];
    for (int k = 0; k < kb; ++k)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int p = 0; p < splits; ++p) s += part[((int64_t)(p * kdim + k) * 3 + c) * N + i];
            U[((int64_t)k * N + i) * 3 + c] = sc * s;
        }
}

// Batched systems: persistent workgroups take items {sys_begin, sys_end,
// target_begin} from an atomic counter; every item covers all sources of its
// system and writes final velocities.
template <typename R, int K, int TPL, int TILE>
__global__ __launch_bounds__(kBlock) void batched_kernel(const R* __restrict__ rec, const int4* __restrict__ items,
                                                         int n_items, unsigned* __restrict__ counter,
                                                         const double* __restrict__ B, double mu0, int64_t Ntot,
                                                         int kb, double* __restrict__ U) {
    __shared__ __attribute__((aligned(16))) R tile[TILE * rec_w<R, K>()];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        const int4 it = items[item];
        Lane<R, K, TPL> L;
        L.load(rec, it.z, it.y, threadIdx.x);
        L.template run<TILE>(rec, it.x, it.y, tile);
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            const int64_t i = (int64_t)it.z + (int64_t)t * kBlock + threadIdx.x;
            if (i >= it.y) continue;
            const double sc = mu0 * B[i];
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (k < kb) U[((int64_t)k * Ntot + i) * 3 + c] = sc * L.total(t, k, c);
        }
    }
}

// ------------------------------------------------------------ symmetric product
//
// Each unordered pair is evaluated once (sym_pairs.h): the target side
// accumulates M_ij f_j, the source side M_ji f_i, which is the same block
// applied with the two off-diagonal wall coefficients exchanged.

// PER: 0 open domain; 1 pseudo-periodic; 2 pseudo-periodic with cell sides
// above 4.5 a, where only the minimum image can overlap its target (every
// other image is at least half a cell away), so the other eight skip the
// overlap branch and their arithmetic can interleave (used in FP64).
template <typename R, int K, int PER = 0>
struct ProductBody {
    static constexpr int KREC = K;
    static constexpr int NQ = 3 * K;
    static constexpr int kUnroll = PER ? 1 : 4;
    // Open domain: two sources per step sharing one overlap branch, so that
    // their arithmetic interleaves (pair2).
    static constexpr bool kDuo = !PER;
    // One source image: target side into acc and, when SYM, source side
    // (transposed block: the two off-diagonal wall coefficients exchanged)
    // into src.
    template <bool SYM>
    __device__ static void image(const SymTarget<R, K>& t, const R* r, R dx, R dy, R dz, R (&acc)[NQ],
                                 R (&src)[NQ]) {
        apply<SYM>(pair_coef<R>(dx, dy, dz, t.z, r[2]), t, r, dx, dy, dz, acc, src);
    }
    // An image that cannot overlap its target (r > 2 a): no overlap branch.
    template <bool SYM>
    __device__ static void far_image(const SymTarget<R, K>& t, const R* r, R dx, R dy, R dz, R (&acc)[NQ],
                                     R (&src)[NQ]) {
        apply<SYM>(pair_fin(pair_pre<R>(dx, dy, dz, t.z, r[2])), t, r, dx, dy, dz, acc, src);
    }
    template <bool SYM>
    __device__ static void apply(PairCoef<R> p, const SymTarget<R, K>& t, const R* r, R dx, R dy, R dz,
                                 R (&acc)[NQ], R (&src)[NQ]) {
        constexpr int PW = pos_slots<R>();
#pragma unroll
        for (int k = 0; k < K; ++k)
            pair_apply<R>(p, dx, dy, dz, r[PW + 3 * k], r[PW + 3 * k + 1], r[PW + 3 * k + 2], acc[3 * k],
                          acc[3 * k + 1], acc[3 * k + 2]);
        if constexpr (SYM) {
            const R x = p.kcp;
            p.kcp = p.kcm;
            p.kcm = x;
#pragma unroll
            for (int k = 0; k < K; ++k)
                pair_apply<R>(p, dx, dy, dz, t.f[k][0], t.f[k][1], t.f[k][2], src[3 * k], src[3 * k + 1],
                              src[3 * k + 2]);
        }
    }
    // Sources ra and rb (open domain): the source sides go to sa and sb.
    template <bool SYM>
    __device__ static void pair2(const SymTarget<R, K>& t, const R* ra, const R* rb, R (&acc)[NQ], R (&sa)[NQ],
                                 R (&sb)[NQ]) {
        R dxa, dya, dza, dxb, dyb, dzb;
        sym_diff(t, ra, dxa, dya, dza);
        sym_diff(t, rb, dxb, dyb, dzb);
        // All four reciprocal square roots are issued before any of their
        // results is used (the empty asm takes them as inputs and outputs),
        // so that their latency overlaps.
        PairGeo<R> ga = pair_geo<R>(dxa, dya, dza, t.z, ra[2]);
        PairGeo<R> gb = pair_geo<R>(dxb, dyb, dzb, t.z, rb[2]);
        __asm__ volatile("" : "+v"(ga.w), "+v"(ga.ir), "+v"(gb.w), "+v"(gb.ir));
        PairPre<R> pa = pair_pre<R>(ga, dza, t.z, ra[2]);
        PairPre<R> pb = pair_pre<R>(gb, dzb, t.z, rb[2]);
        if (__builtin_amdgcn_ballot_w64(pair_near(pa) || pair_near(pb))) {
            __asm__ volatile("" ::: "memory");  // keep this a branch: do not speculate it
            pair_fix(pa);
            pair_fix(pb);
        }
        if constexpr (SYM) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) sa[q] = sb[q] = R(0);
        }
        apply<SYM>(pair_fin(pa), t, ra, dxa, dya, dza, acc, sa);
        apply<SYM>(pair_fin(pb), t, rb, dxb, dyb, dzb, acc, sb);
    }
    // Two images of source r that share one overlap branch, with their four
    // reciprocal square roots issued before any of them is used.
    template <bool SYM>
    __device__ static void image2(const SymTarget<R, K>& t, const R* r, R dxa, R dya, R dxb, R dyb, R dz,
                                  R (&acc)[NQ], R (&src)[NQ]) {
        PairGeo<R> ga = pair_geo<R>(dxa, dya, dz, t.z, r[2]);
        PairGeo<R> gb = pair_geo<R>(dxb, dyb, dz, t.z, r[2]);
        __asm__ volatile("" : "+v"(ga.w), "+v"(ga.ir), "+v"(gb.w), "+v"(gb.ir));
        PairPre<R> pa = pair_pre<R>(ga, dz, t.z, r[2]);
        PairPre<R> pb = pair_pre<R>(gb, dz, t.z, r[2]);
        if (__builtin_amdgcn_ballot_w64(pair_near(pa) || pair_near(pb))) {
            __asm__ volatile("" ::: "memory");  // keep this a branch: do not speculate it
            pair_fix(pa);
            pair_fix(pb);
        }
        apply<SYM>(pair_fin(pa), t, r, dxa, dya, dz, acc, src);
        apply<SYM>(pair_fin(pb), t, r, dxb, dyb, dz, acc, src);
    }
    template <bool SYM>
    __device__ static void pair(const SymTarget<R, K>& t, const R* r, R (&acc)[NQ], R (&src)[NQ],
                                const Box<R>& box) {
        R dx, dy, dz;
        sym_diff(t, r, dx, dy, dz);
        if constexpr (SYM) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) src[q] = R(0);
        }
        if constexpr (!PER) {
            image<SYM>(t, r, dx, dy, dz, acc, src);
        } else {
            // Pseudo-periodic domain: the source's minimum image (records
            // are wrapped into the cell, so the shift is 0 or one cell) and
            // the 8 periodic images around it.
            const R nx = rint_(dx * box.ilx), ny = rint_(dy * box.ily);
            dx = fma_(-nx, box.lxl, fma_(-nx, box.lxh, dx));
            dy = fma_(-ny, box.lyl, fma_(-ny, box.lyh, dy));
            // image k: shift (k / 3 - 1, k % 3 - 1) cells
            auto shifted = [&](int k, R& ex, R& ey) {
                const int sx = k / 3 - 1, sy = k % 3 - 1;
                ex = sx == 0 ? dx : sx < 0 ? dx - box.lx : dx + box.lx;
                ey = sy == 0 ? dy : sy < 0 ? dy - box.ly : dy + box.ly;
            };
            if constexpr (PER == 1) {
                // images in pairs, each pair sharing one overlap branch
#pragma unroll
                for (int k = 0; k < 8; k += 2) {
                    R ea, fa, eb, fb;
                    shifted(k, ea, fa);
                    shifted(k + 1, eb, fb);
                    image2<SYM>(t, r, ea, fa, eb, fb, dz, acc, src);
                }
                R e8, f8;
                shifted(8, e8, f8);
                image<SYM>(t, r, e8, f8, dz, acc, src);
                return;
            }
#pragma unroll
            for (int sx = -1; sx <= 1; ++sx)
#pragma unroll
                for (int sy = -1; sy <= 1; ++sy) {
                    const R ex = sx == 0 ? dx : sx < 0 ? dx - box.lx : dx + box.lx;
                    const R ey = sy == 0 ? dy : sy < 0 ? dy - box.ly : dy + box.ly;
                    if (PER == 2 && (sx != 0 || sy != 0))
                        far_image<SYM>(t, r, ex, ey, dz, acc, src);
                    else
                        image<SYM>(t, r, ex, ey, dz, acc, src);
                }
        }
    }
};

// kEpiParts threads per (blob, output component q = 3k + c): each adds its
// share of the partials (sym_gather), then the shares are added in a fixed
// order.  Blocks cover 64 consecutive blobs (coalesced partial reads).
constexpr int kEpiParts = 8;
template <typename R>
__global__ __launch_bounds__(64 * kEpiParts) void sym_epilogue(const double* __restrict__ tpart,
                                                               const R* __restrict__ spart,
                                                               const double* __restrict__ B, int64_t N, int ng, int C,
                                                               int Hmax, int nseg, int K, int G, double mu0,
                                                               double* __restrict__ U,
                                                               const double* __restrict__ pos, double inv_a) {
    __shared__ double red[kEpiParts][64];
    const int x = threadIdx.x & 63, u = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + x;
    const int q = blockIdx.y;
    red[u][x] = i < N ? sym_gather<R>(tpart, spart, i, ng, C, Hmax, 3 * K, q, G, u, kEpiParts, nseg) : 0.0;
    __syncthreads();
    if (u != 0 || i >= N) return;
    double s = red[0][x];
#pragma unroll
    for (int v = 1; v < kEpiParts; ++v) s += red[v][x];
    double b;
    if (B) {
        b = B[i];
    } else {  // records formed in the pair kernel: B from the position
        const double z = pos[3 * i + 2] * inv_a;
        b = z < 1.0 ? z : 1.0;
    }
    U[((int64_t)(q / 3) * N + i) * 3 + q % 3] = mu0 * b * s;
}

// ps: the kernel forms its records from ps (groups of 64 only); otherwise
// they are read from rec.
template <typename R, int K, int PER>
hipError_t launch_sym_t(const R* rec, const SymPlan& sp, int ipw, double* tpart, R* spart, const Box<R>& box,
                        hipStream_t st, const PackSrc* ps = nullptr) {
    const dim3 grid((unsigned)((int64_t)sp.ng * sp.C * sp.nseg));
    const PackSrc p0 = ps ? *ps : PackSrc{};
    if (ps && sp.G != 64) return hipErrorInvalidValue;
    if (sp.G == 64 && sp.ns == 4) {
        if (ps)
            hipLaunchKernelGGL((sym_kernel<R, ProductBody<R, K, PER>, 1, 4, true>), grid, dim3(256), 0, st, rec, sp.ng,
                               sp.C, ipw, sp.Hmax, sp.nseg, tpart, spart, box, p0);
        else
            hipLaunchKernelGGL((sym_kernel<R, ProductBody<R, K, PER>, 1, 4>), grid, dim3(256), 0, st, rec, sp.ng, sp.C,
                               ipw, sp.Hmax, sp.nseg, tpart, spart, box, p0);
    } else if (sp.G == 64) {
        if (ps)
            hipLaunchKernelGGL((sym_kernel<R, ProductBody<R, K, PER>, 1, 1, true>), grid, dim3(64), 0, st, rec, sp.ng,
                               sp.C, ipw, sp.Hmax, sp.nseg, tpart, spart, box, p0);
        else
            hipLaunchKernelGGL((sym_kernel<R, ProductBody<R, K, PER>, 1>), grid, dim3(64), 0, st, rec, sp.ng, sp.C,
                               ipw, sp.Hmax, sp.nseg, tpart, spart, box, p0);
    } else {
        hipLaunchKernelGGL((sym_kernel<R, ProductBody<R, K, PER>, 4>), grid, dim3(256), 0, st, rec, sp.ng, sp.C, ipw,
                           sp.Hmax, sp.nseg, tpart, spart, box, p0);
    }
    return hipGetLastError();
}

// Kernel-side cell description in units of a (zeros for the open domain).
template <typename R>
Box<R> make_box(const Domain& dom, double a) {
    Box<R> b{};
    if (!dom.periodic()) return b;
    auto split = [](double L, R& hi, R& lo) {
        int e;
        std::frexp(L, &e);
        const double h = std::ldexp(std::nearbyint(std::ldexp(L, 12 - e)), e - 12);  // 12 significant bits
        hi = (R)h;
        lo = (R)(L - h);
    };
    const double lx = dom.lx / a, ly = dom.ly / a;
    b.lx = (R)lx;
    b.ly = (R)ly;
    split(lx, b.lxh, b.lxl);
    split(ly, b.lyh, b.lyl);
    b.ilx = (R)(1.0 / lx);
    b.ily = (R)(1.0 / ly);
    return b;
}

__global__ void zero_u32(unsigned* p) { *p = 0u; }

// ------------------------------------------------------------ dispatch

template <typename R, int K, int TPL, int TILE>
hipError_t launch_pair_t(const R* rec, int64_t N, int splits, int64_t chunk, double* part, int64_t nblocks,
                         hipStream_t st) {
    hipLaunchKernelGGL((pair_kernel<R, K, TPL, TILE>), dim3((unsigned)nblocks), dim3(kBlock), 0, st, rec, N, splits,
                       chunk, part);
    return hipGetLastError();
}

template <typename R, int K, int TPL, int TILE>
hipError_t launch_batched_t(const R* rec, const int4* items, int n_items, unsigned* counter, const double* B,
                            double mu0, int64_t Ntot, int kb, double* U, int grid, hipStream_t st) {
    hipLaunchKernelGGL((batched_kernel<R, K, TPL, TILE>), dim3(grid), dim3(kBlock), 0, st, rec, items, n_items,
                       counter, B, mu0, Ntot, kb, U);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t launch_mat_t(const void* rec, int64_t N, int splits, int64_t chunk, double* part, int64_t nblocks,
                        hipStream_t st) {
    hipLaunchKernelGGL((mat_pair_kernel<R, K>), dim3((unsigned)nblocks), dim3(kBlock), 0, st, (const R*)rec, N, splits,
                       chunk, part);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t launch_mat_batched_t(const void* rec, const int4* items, int n_items, unsigned* counter,
                                const double* B, double mu0, int64_t Ntot, int kb, double* U, int grid,
                                hipStream_t st) {
    hipLaunchKernelGGL((mat_batched_kernel<R, K>), dim3(grid), dim3(kBlock), 0, st, (const R*)rec, items, n_items,
                       counter, B, mu0, Ntot, kb, U);
    return hipGetLastError();
}

// The matrix-core launches for a precision and a block of 8 or 16.
hipError_t launch_mat(int prec, int K, const void* rec, int64_t N, int splits, int64_t chunk, double* part,
                      int64_t nblocks, hipStream_t st) {
    if (prec == RPYW_FP32C)
        return K == 16 ? launch_mat_t<float, 16>(rec, N, splits, chunk, part, nblocks, st)
                       : launch_mat_t<float, 8>(rec, N, splits, chunk, part, nblocks, st);
    return K == 16 ? launch_mat_t<double, 16>(rec, N, splits, chunk, part, nblocks, st)
                   : launch_mat_t<double, 8>(rec, N, splits, chunk, part, nblocks, st);
}

hipError_t launch_mat_batched(int prec, int K, const void* rec, const int4* items, int n_items, unsigned* counter,
                              const double* B, double mu0, int64_t Ntot, int kb, double* U, int grid,
                              hipStream_t st) {
    if (prec == RPYW_FP32C)
        return K == 16 ? launch_mat_batched_t<float, 16>(rec, items, n_items, counter, B, mu0, Ntot, kb, U, grid, st)
                       : launch_mat_batched_t<float, 8>(rec, items, n_items, counter, B, mu0, Ntot, kb, U, grid, st);
    return K == 16 ? launch_mat_batched_t<double, 16>(rec, items, n_items, counter, B, mu0, Ntot, kb, U, grid, st)
                   : launch_mat_batched_t<double, 8>(rec, items, n_items, counter, B, mu0, Ntot, kb, U, grid, st);
}

// Expand (K, TPL, TILE) runtime values into template instantiations.
#define RPYW_DISPATCH(R, K, TPL, TILE, FN, ...)                                   \
    [&]() -> hipError_t {                                                         \
        auto tiles = [&](auto kc, auto tc) -> hipError_t {                        \
            constexpr int KK = decltype(kc)::value;                               \
            constexpr int TT = decltype(tc)::value;                               \
            if ((TILE) == 64) return FN<R, KK, TT, 64>(__VA_ARGS__);              \
            return FN<R, KK, TT, 256>(__VA_ARGS__);                               \
        };                                                                        \
        auto tpls = [&](auto kc) -> hipError_t {                                  \
            if ((TPL) == 2) return tiles(kc, std::integral_constant<int, 2>{});   \
            return tiles(kc, std::integral_constant<int, 1>{});                   \
        };                                                                        \
        auto one = [&](auto kc) -> hipError_t {                                   \
            return tiles(kc, std::integral_constant<int, 1>{});                   \
        };                                                                        \
        switch (K) {                                                              \
            case 1: return tpls(std::integral_constant<int, 1>{});                \
            case 2: return tpls(std::integral_constant<int, 2>{});                \
            case 4: return tpls(std::integral_constant<int, 4>{});                \
            case 8: return one(std::integral_constant<int, 8>{});                 \
            default:                                                              \
                if constexpr (sizeof(R) == 8) return one(std::integral_constant<int, 8>{}); \
                else return one(std::integral_constant<int, 16>{});               \
        }                                                                         \
    }()

int pow2ceil(int k) {
    int p = 1;
    while (p < k) p <<= 1;
    return p;
}

// RHS block width of the kernel instantiation that serves kb right-hand
// sides (on the vector units FP64 stops at 8: wider blocks do not fit the
// register file; the matrix-core kernel takes 16 in both precisions).
int kernel_k(int kb, int prec, int mat) {
    return std::min(pow2ceil(kb), (prec == RPYW_FP32C || mat) ? 16 : 8);
}

// The launch shape the dispatch actually instantiates: blocks of 8 or more
// right-hand sides run one target per lane, tiles are 64 or 256.
Shape normalized(Shape s, int K, int prec) {
    (void)prec;
    s.mat = (s.mat && K >= 8) ? 1 : 0;
    if (K >= 8) s.tpl = 1;
    if (K > 4) s.sym = 0;
    if (s.ipw < 1) s.ipw = 4;
    s.tpl = s.tpl == 2 ? 2 : 1;
    s.tile = s.tile == 64 ? 64 : 256;
    return s;
}

double mu0_of(double a, double eta) { return 1.0 / (6.0 * M_PI * eta * a); }

}  // namespace

// ------------------------------------------------------------ host side

SymPlan sym_plan(int64_t N, int prec, int K, int ipw, int G) {
    SymPlan s{};
    s.G = G == 64 ? 64 : 256;
    s.ng = (int)((N + s.G - 1) / s.G);
    s.Hmax = s.ng / 2;
    if (ipw < 1) ipw = 1;
    s.C = (s.Hmax + 1 + ipw - 1) / ipw;
    // Segments: enough work items to give every SIMD several (independent
    // of ipw, so that the workspace bound taken at ipw 1 holds).
    const int64_t items = (int64_t)s.ng * (s.Hmax + 1);
    // Groups of 64 split the passes of few items over 4 waves of one
    // workgroup first (their sums meet in LDS), and over workgroups (each
    // with partials of its own) only when there are fewer than half as many
    // waves as wanted.
    s.ns = (s.G == 64 && items < kSymItemsMin) ? 4 : 1;
    const int64_t want = s.ns > 1 ? kSymItemsMin / 2 : kSymItemsMin;
    s.nseg = 1;
    while (s.nseg < 4 && items * s.ns * s.nseg < want) s.nseg *= 2;
    if (s.G == 64) sym_split_override(&s.ns, &s.nseg);
    const size_t npad = (size_t)s.ng * s.G;
    s.rec_bytes = align_up(npad * rec_width(prec, K) * real_size(prec)) + align_up(npad * sizeof(double));
    s.tpart_bytes = align_up((size_t)s.ng * s.C * s.nseg * 3 * K * s.G * sizeof(double));
    s.spart_bytes = align_up((size_t)s.ng * (s.Hmax + 1) * s.nseg * 3 * K * s.G * real_size(prec));
    s.ok = K <= 4 && s.spart_bytes <= kSymPartialMaxBytes && s.tpart_bytes <= kSymPartialMaxBytes &&
           (s.G == 256 || N <= kSym64MaxN);
    return s;
}

void split_plan(int64_t N, int tpl, int* splits, int64_t* chunk) {
    const int64_t ntb = (N + (int64_t)kBlock * tpl - 1) / ((int64_t)kBlock * tpl);
    const int64_t want_wg = 2048;
    int64_t s = (want_wg + ntb - 1) / ntb;
    const int64_t max_s = std::max<int64_t>(1, N / 64);
    if (s > max_s) s = max_s;
    if (s > 8) s = (s + 7) / 8 * 8;
    if (s < 1) s = 1;
    int64_t c = (N + s - 1) / s;
    s = (N + c - 1) / c;
    *splits = (int)s;
    *chunk = c;
}

// Source chunks of the matrix-core kernel: workgroups of 64 targets, enough
// of them for several rounds of five per CU (the tail of the last round
// then costs little), chunks of at least 256 sources.
void mat_split_plan(int64_t N, int* splits, int64_t* chunk) {
    const int64_t ntb = (N + kMatTargets - 1) / kMatTargets;
    const int64_t want_wg = 8192;
    int64_t s = (want_wg + ntb - 1) / ntb;
    const int64_t max_s = std::max<int64_t>(1, N / 256);
    if (s > max_s) s = max_s;
    if (s > 8) s = (s + 7) / 8 * 8;
    if (s < 1) s = 1;
    int64_t c = (N + s - 1) / s;
    s = (N + c - 1) / c;
    *splits = (int)s;
    *chunk = c;
}

size_t product_ws_bytes(int64_t N, int prec, int kblk) {
    int s1, s2, s3 = 1;
    int64_t c;
    split_plan(N, 1, &s1, &c);
    split_plan(N, 2, &s2, &c);
    if (kblk >= 8) mat_split_plan(N, &s3, &c);
    const int smax = std::max(std::max(s1, s2), s3);
    size_t b = align_up((size_t)N * rec_width(prec, kblk) * real_size(prec));
    b += align_up((size_t)N * sizeof(double));
    b += align_up((size_t)smax * kblk * 3 * N * sizeof(double));
    size_t sb = 0;
    for (int K = 1; K <= std::min(kblk, 4); K <<= 1)
        for (int G : {256, 64}) {
            const SymPlan sp = sym_plan(N, prec, K, 1, G);
            if (sp.ok) sb = std::max(sb, sp.rec_bytes + sp.tpart_bytes + sp.spart_bytes);
        }
    return std::max(b, sb) + 8 * kAlign;
}

namespace {

int sym_pass(const double* pos, const double* F, double* U, int64_t N, int kb, int K, double a, double eta, int prec,
             const SymPlan& sp, int ipw, Arena& ar, hipStream_t st, const Domain& dom = Domain{}) {
    const size_t mark = ar.used;
    double* tpart = (double*)ar.take(sp.tpart_bytes);
    void* spart = ar.take(sp.spart_bytes);
    if (!tpart || !spart) {
        ar.used = mark;
        return RPYW_ENOMEM;
    }
    // Groups of 64 (small problems): the pair kernel forms the records
    // itself, two launches per product; otherwise the records are packed
    // once by their own kernel.
    const bool fused = sp.G == 64;
    const PackSrc ps{pos, F, N, kb, 1.0 / a, dom.lx / a, dom.ly / a};
    void* rec = nullptr;
    double* B = nullptr;
    int rc = RPYW_OK;
    if (!fused) {
        const int rw = rec_width(prec, K);
        const int64_t npad = (int64_t)sp.ng * sp.G;
        rec = ar.take((size_t)npad * rw * real_size(prec));
        B = (double*)ar.take((size_t)npad * sizeof(double));
        if (!rec || !B) {
            ar.used = mark;
            return RPYW_ENOMEM;
        }
        rc = sym_pack(pos, F, N, kb, K, prec, sp, a, dom, rec, B, st);
    }
    if (rc == RPYW_OK) {
        hipEvent_t ev = nullptr;
        profile_begin(st, &ev);
        rc = sym_launch(rec, sp, ipw, K, prec, a, dom, tpart, spart, st, fused ? &ps : nullptr);
        if (rc == RPYW_OK) {
            profile_end(st, ev, (dom.periodic() ? 9.0 : 1.0) * (double)kb * (double)N * (double)N);
            rc = sym_finish(tpart, spart, B, N, kb, K, prec, sp, mu0_of(a, eta), U, st, pos, 1.0 / a);
        }
    }
    ar.used = mark;
    return rc;
}

}  // namespace

int sym_pack(const double* pos, const double* F, int64_t N, int kb, int K, int prec, const SymPlan& sp, double a,
             const Domain& dom, void* rec, double* B, hipStream_t st) {
    const int rw = rec_width(prec, K);
    const int64_t npad = (int64_t)sp.ng * sp.G;
    const unsigned g1 = (unsigned)((npad + kBlock - 1) / kBlock);
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(pack_kernel<float>, dim3(g1), dim3(kBlock), 0, st, pos, F, N, kb, rw, 1.0 / a, (float*)rec, B,
                           nullptr, dom.lx / a, dom.ly / a, npad);
    else
        hipLaunchKernelGGL(pack_kernel<double>, dim3(g1), dim3(kBlock), 0, st, pos, F, N, kb, rw, 1.0 / a,
                           (double*)rec, B, nullptr, dom.lx / a, dom.ly / a, npad);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int sym_launch(const void* rec, const SymPlan& sp, int ipw, int K, int prec, double a, const Domain& dom,
               double* tpart, void* spart, hipStream_t st, const PackSrc* ps) {
    auto go = [&](auto Rt, auto Kc) -> hipError_t {
        using R = decltype(Rt);
        constexpr int KK = decltype(Kc)::value;
        if (dom.periodic()) {
            if constexpr (KK == 1) {
                // FP64 only: in FP32 the branch-free far images measured
                // 4-7% slower, in FP64 up to 10% faster
                if constexpr (sizeof(R) == 8)
                    if (std::min(dom.lx, dom.ly) > 4.5 * a)
                        return launch_sym_t<R, 1, 2>((const R*)rec, sp, ipw, tpart, (R*)spart, make_box<R>(dom, a),
                                                     st, ps);
                return launch_sym_t<R, 1, 1>((const R*)rec, sp, ipw, tpart, (R*)spart, make_box<R>(dom, a), st, ps);
            }
            return hipErrorInvalidValue;
        }
        return launch_sym_t<R, KK, 0>((const R*)rec, sp, ipw, tpart, (R*)spart, Box<R>{}, st, ps);
    };
    hipError_t e;
    if (prec == RPYW_FP32C)
        e = K == 1 ? go(0.f, std::integral_constant<int, 1>{})
                   : K == 2 ? go(0.f, std::integral_constant<int, 2>{}) : go(0.f, std::integral_constant<int, 4>{});
    else
        e = K == 1 ? go(0.0, std::integral_constant<int, 1>{})
                   : K == 2 ? go(0.0, std::integral_constant<int, 2>{}) : go(0.0, std::integral_constant<int, 4>{});
    return e == hipSuccess ? RPYW_OK : RPYW_EHIP;
}

int sym_finish(const double* tpart, const void* spart, const double* B, int64_t N, int kb, int K, int prec,
               const SymPlan& sp, double mu0, double* U, hipStream_t st, const double* pos, double inv_a) {
    if (!B && !pos) return RPYW_EINVAL;
    const dim3 ge((unsigned)((N + 63) / 64), (unsigned)(3 * kb));
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(sym_epilogue<float>, ge, dim3(64 * kEpiParts), 0, st, tpart, (const float*)spart, B, N,
                           sp.ng, sp.C, sp.Hmax, sp.nseg, K, sp.G, mu0, U, pos, inv_a);
    else
        hipLaunchKernelGGL(sym_epilogue<double>, ge, dim3(64 * kEpiParts), 0, st, tpart, (const double*)spart, B, N,
                           sp.ng, sp.C, sp.Hmax, sp.nseg, K, sp.G, mu0, U, pos, inv_a);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}

int product_pass(const double* pos, const double* F, double* U, int64_t N, int kb, double a, double eta, int prec,
                 Shape sh, Arena& ar, hipStream_t st) {
    const size_t mark = ar.used;
    const int K = kernel_k(kb, prec, sh.mat);
    if (kb < 1 || kb > K) return RPYW_EINVAL;
    sh = normalized(sh, K, prec);
    if (sh.sym && K <= 4) {
        SymPlan sp = sym_plan(N, prec, K, sh.ipw, sym_group(sh.sym));
        if (!sp.ok && sp.G == 64) sp = sym_plan(N, prec, K, sh.ipw, 256);
        if (sp.ok) return sym_pass(pos, F, U, N, kb, K, a, eta, prec, sp, sh.ipw, ar, st);
    }
    const int rw = rec_width(prec, K);
    void* rec = ar.take((size_t)N * rw * real_size(prec));
    double* B = (double*)ar.take((size_t)N * sizeof(double));
    int splits;
    int64_t chunk;
    if (sh.mat)
        mat_split_plan(N, &splits, &chunk);
    else
        split_plan(N, sh.tpl, &splits, &chunk);
    double* part = (double*)ar.take((size_t)splits * K * 3 * N * sizeof(double));
    if (!rec || !B || !part) {
        ar.used = mark;
        return RPYW_ENOMEM;
    }
    const unsigned g1 = (unsigned)((N + kBlock - 1) / kBlock);
    if (prec == RPYW_FP32C)
        hipLaunchKernelGGL(pack_kernel<float>, dim3(g1), dim3(kBlock), 0, st, pos, F, N, kb, rw, 1.0 / a, (float*)rec,
                           B, nullptr, 0.0, 0.0, N);
    else
        hipLaunchKernelGGL(pack_kernel<double>, dim3(g1), dim3(kBlock), 0, st, pos, F, N, kb, rw, 1.0 / a,
                           (double*)rec, B, nullptr, 0.0, 0.0, N);
    RPYW_HIP(hipGetLastError());
    const int span = sh.mat ? kMatTargets : kBlock * sh.tpl;
    const int64_t ntb = (N + span - 1) / span;
    const int64_t nblocks = ntb * splits;
    hipEvent_t ev = nullptr;
    profile_begin(st, &ev);
    hipError_t e;
    if (sh.mat)
        e = launch_mat(prec, K, rec, N, splits, chunk, part, nblocks, st);
    else if (prec == RPYW_FP32C)
        e = RPYW_DISPATCH(float, K, sh.tpl, sh.tile, launch_pair_t, (const float*)rec, N, splits, chunk, part, nblocks,
                          st);
    else
        e = RPYW_DISPATCH(double, K, sh.tpl, sh.tile, launch_pair_t, (const double*)rec, N, splits, chunk, part,
                          nblocks, st);
    if (e != hipSuccess) return RPYW_EHIP;
    profile_end(st, ev, (double)kb * (double)N * (double)N);
    hipLaunchKernelGGL(epilogue_kernel, dim3(g1), dim3(kBlock), 0, st, part, B, N, K, kb, splits, mu0_of(a, eta), U);
    RPYW_HIP(hipGetLastError());
    ar.used = mark;
    return RPYW_OK;
}

int products(const double* pos, const double* F, double* U, int64_t N, int k, double a, double eta, int prec,
             Arena& ar, hipStream_t st, const Domain& dom) {
    if (dom.periodic()) {
        // Always symmetric (one right-hand side per pass): groups of 64
        // unless the shape asks for groups of 256.
        const Shape sh = tuned_shape(N, 1, prec);
        SymPlan sp = sym_plan(N, prec, 1, sh.ipw, sh.sym == 1 ? 256 : 64);
        if (!sp.ok) sp = sym_plan(N, prec, 1, sh.ipw, 256);
        if (!sp.ok) return RPYW_ENOMEM;
        for (int k0 = 0; k0 < k; ++k0) {
            const int rc = sym_pass(pos, F + (size_t)k0 * N * 3, U + (size_t)k0 * N * 3, N, 1, 1, a, eta, prec, sp,
                                    sh.ipw, ar, st, dom);
            if (rc != RPYW_OK) return rc;
        }
        return RPYW_OK;
    }
    Shape sh = tuned_shape(N, k, prec);
    if (prec != RPYW_FP32C && !sh.mat) sh.kblk = std::min(sh.kblk, 8);  // e.g. RPYW_RHS_WIDTH=16 on the vector units
    for (int k0 = 0; k0 < k; k0 += sh.kblk) {
        const int kb = std::min(sh.kblk, k - k0);
        const int rc = product_pass(pos, F + (size_t)k0 * N * 3, U + (size_t)k0 * N * 3, N, kb, a, eta, prec, sh, ar,
                                    st);
        if (rc != RPYW_OK) return rc;
    }
    return RPYW_OK;
}

// ------------------------------------------------------------ batched

size_t batched_ws_bytes(int64_t Ntot, int S, int k, int prec) {
    const int kb = kernel_k(std::max(k, 1), prec, 1);  // the widest the batched kernels take
    size_t b = align_up((size_t)Ntot * rec_width(prec, kb) * real_size(prec));
    b += align_up((size_t)Ntot * sizeof(double));
    const size_t max_items = (size_t)(Ntot / kMatTargets) + (size_t)S + 1;  // items of 64 or more targets
    b += align_up(max_items * sizeof(int4));
    b += kAlign;  // counter
    return b + 4 * kAlign;
}

int batched_products(const double* pos, const int64_t* sys_offsets, int S, const double* F, double* U, int k,
                     double a, double eta, int prec, Arena& ar, hipStream_t st) {
    const int64_t Ntot = sys_offsets[S];
    int64_t nmax = 0;
    for (int s = 0; s < S; ++s) nmax = std::max(nmax, sys_offsets[s + 1] - sys_offsets[s]);
    // The batched kernel is the plain one, with the widest RHS block (one
    // pass over the sources per item): the shapes tuned for products of one
    // system (a symmetric kernel, or narrower blocks that fill the GPU with a
    // single system) do not carry over to a persistent launch over many; the
    // RPYW_TILE / RPYW_RHS_WIDTH overrides still apply.
    Shape sh = default_shape(nmax, k, prec);
    sh.sym = 0;
    sh = apply_env_overrides(sh);
    sh = normalized(sh, kernel_k(sh.kblk, prec, sh.mat), prec);
    // Work list in LPT order: systems by decreasing size, then their tiles.
    std::vector<int> order(S);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return sys_offsets[x + 1] - sys_offsets[x] > sys_offsets[y + 1] - sys_offsets[y];
    });
    const int span = sh.mat ? kMatTargets : kBlock * sh.tpl;
    std::vector<int4> items;
    for (int s : order) {
        const int b0 = (int)sys_offsets[s], b1 = (int)sys_offsets[s + 1];
        for (int t = b0; t < b1; t += span) items.push_back(make_int4(b0, b1, t, 0));
    }
    const size_t mark = ar.used;
    const int K = kernel_k(sh.kblk, prec, sh.mat);
    if (sh.kblk > K) return RPYW_EINVAL;
    const int rw = rec_width(prec, K);
    void* rec = ar.take((size_t)Ntot * rw * real_size(prec));
    double* B = (double*)ar.take((size_t)Ntot * sizeof(double));
    int4* ditems = (int4*)ar.take(items.size() * sizeof(int4));
    unsigned* counter = (unsigned*)ar.take(sizeof(unsigned));
    if (!rec || !B || !ditems || !counter) {
        ar.used = mark;
        return RPYW_ENOMEM;
    }
    int rc = stage_upload(items.data(), items.size() * sizeof(int4), ditems, st);
    if (rc != RPYW_OK) return rc;
    int dev = 0, ncu = 256;
    RPYW_HIP(hipGetDevice(&dev));
    RPYW_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = sh.mat ? (prec == RPYW_FP32C ? mat_batched_waves<float>() : mat_batched_waves<double>()) : 4;
    const int grid = (int)std::min<size_t>(items.size(), (size_t)ncu * per_cu);
    const unsigned g1 = (unsigned)((Ntot + kBlock - 1) / kBlock);
    const double m0 = mu0_of(a, eta);
    double pairs = 0.0;
    for (int s = 0; s < S; ++s) {
        const double n = (double)(sys_offsets[s + 1] - sys_offsets[s]);
        pairs += n * n;
    }
    for (int k0 = 0; k0 < k; k0 += sh.kblk) {
        const int kb = std::min(sh.kblk, k - k0);
        const double* Fk = F + (size_t)k0 * Ntot * 3;
        double* Uk = U + (size_t)k0 * Ntot * 3;
        if (prec == RPYW_FP32C)
            hipLaunchKernelGGL(pack_kernel<float>, dim3(g1), dim3(kBlock), 0, st, pos, Fk, Ntot, kb, rw, 1.0 / a,
                               (float*)rec, B, nullptr, 0.0, 0.0, Ntot);
        else
            hipLaunchKernelGGL(pack_kernel<double>, dim3(g1), dim3(kBlock), 0, st, pos, Fk, Ntot, kb, rw, 1.0 / a,
                               (double*)rec, B, nullptr, 0.0, 0.0, Ntot);
        RPYW_HIP(hipGetLastError());
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(1), 0, st, counter);
        RPYW_HIP(hipGetLastError());
        hipEvent_t ev = nullptr;
        profile_begin(st, &ev);
        hipError_t e;
        if (sh.mat)
            e = launch_mat_batched(prec, K, rec, ditems, (int)items.size(), counter, B, m0, Ntot, kb, Uk, grid, st);
        else if (prec == RPYW_FP32C)
            e = RPYW_DISPATCH(float, K, sh.tpl, sh.tile, launch_batched_t, (const float*)rec, ditems,
                              (int)items.size(), counter, B, m0, Ntot, kb, Uk, grid, st);
        else
            e = RPYW_DISPATCH(double, K, sh.tpl, sh.tile, launch_batched_t, (const double*)rec, ditems,
                              (int)items.size(), counter, B, m0, Ntot, kb, Uk, grid, st);
        if (e != hipSuccess) return RPYW_EHIP;
        profile_end(st, ev, kb * pairs);
    }
    ar.used = mark;
    return RPYW_OK;
}

}  // namespace rpyw
