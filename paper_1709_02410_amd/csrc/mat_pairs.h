// Multi-RHS products on the matrix cores (FP32C blocks of 8 or 16
// right-hand sides): the product and batched kernels that pair_kernels.hip
// launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "pair_math.h"
#include "records.h"
#include "rpyw_internal.h"

namespace rpyw {

// With a block of K >= 8 right-hand sides the product is a dense contraction:
// u_i = sum_j M_ij F_j, F_j the 3 x K block of source j's forces.  The vector
// units form each 3 x 3 block M_ij once (the pair geometry and its wall
// coefficients); the matrix cores contract the blocks with F, one
// v_mfma_f32_16x16x4f32 per block entry (c, d) and step of 4 sources:
//   D_c[t][k] += sum_{s < 4} M_cd(t, s) F_d(s, k),  16 targets t x 16 RHS k.
// A wave holds 16 targets.  In each step lane l evaluates the pair (target
// l % 16, source l / 16): its nine block entries are the A operands (row t =
// l % 16, column s = l / 16) of the step's nine instructions, and component d
// of right-hand side l % 16 of source l / 16 is the B operand (row s, column
// k) of the three instructions of column d.  Accumulator c of lane l holds
// velocity component c of targets 4 (l / 16) + v, v < 4, for right-hand side
// l % 16.  The instructions sum in FP32 within a tile of sources; after each
// tile the sums are folded into TwoSum (hi, lo) pairs, as on the vector
// path.  Right-hand sides k >= K (K = 8) contract zero forces.
// FP64 products take v_mfma_f64_16x16x4f64, with the same A and B lane
// layout; its accumulator v of lane l holds target l / 16 + 4 v instead
// (checked on the GPU by a probe product, as the FP32 layout).  They sum in
// FP64 (no compensation); their records carry no low position parts.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mat_fma(float a, float b, mf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ md4 mat_fma(double a, double b, md4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kMatWaveTargets = 16;
constexpr int kMatTargets = kMatWaveTargets * (kBlock / 64);  // per workgroup
// sources per LDS tile (FP32: 28 KB at 16 RHS; FP64: 26 KB)
template <typename R>
constexpr int mat_tile() {
    return sizeof(R) == 4 ? 128 : 64;
}

template <typename R, int K>
struct MatLane {
    static constexpr bool F32 = sizeof(R) == 4;
    static constexpr int RW = rec_w<R, K>();
    static constexpr int PW = pos_slots<R>();
    static constexpr int TILE = mat_tile<R>();
    using Acc = std::conditional_t<F32, mf4, md4>;
    R x, y, z, xl, yl;  // target l % 16 of the wave's 16 (xl, yl: FP32 low parts)
    Acc acc[3];
    R hi[3][4], lo[3][4];  // FP32 compensated sums

    __device__ void load(const R* __restrict__ rec, int64_t first, int64_t last) {
        int64_t i = first + kMatWaveTargets * (threadIdx.x >> 6) + (threadIdx.x & 15);
        if (i >= last) i = last - 1;
        const R* r = rec + i * RW;
        x = r[0];
        y = r[1];
        z = r[2];
        xl = F32 ? r[3] : R(0);
        yl = F32 ? r[4] : R(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hi[c][v] = R(0);
                lo[c][v] = R(0);
            }
        }
    }

    // Sum over sources [s0, s1) staged through the LDS tile.  Slots past the
    // last source of a tile, up to the next multiple of 4, hold force-free
    // blobs far from everything (their blocks are finite, their forces 0).
    __device__ void run(const R* __restrict__ rec, int64_t s0, int64_t s1, R* tile) {
        const int q = (threadIdx.x >> 4) & 3;  // source of the step
        const int k = threadIdx.x & 15;        // right-hand side
        const int kf = k < K ? k : 0;
        const R fscale = k < K ? R(1) : R(0);
        for (int64_t t0 = s0; t0 < s1; t0 += TILE) {
            const int n = (int)((s1 - t0) < TILE ? (s1 - t0) : TILE);
            const int n4 = (n + 3) & ~3;
            __syncthreads();
            const R* g = rec + t0 * RW;
            for (int e = threadIdx.x; e < n * RW; e += kBlock) tile[e] = g[e];
            for (int e = n * RW + threadIdx.x; e < n4 * RW; e += kBlock) {
                const int o = e % RW;
                tile[e] = o < 2 ? R(1e6) : (o == 2 ? R(1) : R(0));
            }
            __syncthreads();
            // Software pipeline: the vector units form the block of step
            // j + 4 while the matrix cores contract step j (the last step of
            // a tile forms a copy of itself, which is not used).  The
            // scheduling groups interleave the two: six contractions go with
            // the tile reads and distances of the next step, before its
            // overlap branch, three with its wall coefficients after it.
            // Without them the loop ran up to 18% slower at 1e5 blobs (on
            // some MI355X units; the same on others).
            PairPre<R> pp;
            R dx, dy, dz, fn[3];
            front(tile, 0, q, kf, fscale, pp, dx, dy, dz, fn);
            PairBlock<R> m = back(pp, dx, dy, dz);
            R f[3] = {fn[0], fn[1], fn[2]};
            for (int j = 0; j < n4; j += 4) {
                front(tile, j + 4 < n4 ? j + 4 : j, q, kf, fscale, pp, dx, dy, dz, fn);
                acc[0] = mat_fma(m.xx, f[0], acc[0]);
                acc[1] = mat_fma(m.xy, f[0], acc[1]);
                acc[2] = mat_fma(m.zx, f[0], acc[2]);
                acc[0] = mat_fma(m.xy, f[1], acc[0]);
                acc[1] = mat_fma(m.yy, f[1], acc[1]);
                acc[2] = mat_fma(m.zy, f[1], acc[2]);
                __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);  // LDS reads
                for (int i = 0; i < 6; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);  // seven VALU
                }
                const PairBlock<R> mn = back(pp, dx, dy, dz);
                acc[0] = mat_fma(m.xz, f[2], acc[0]);
                acc[1] = mat_fma(m.yz, f[2], acc[1]);
                acc[2] = mat_fma(m.zz, f[2], acc[2]);
                for (int i = 0; i < 3; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                }
                m = mn;
                f[0] = fn[0];
                f[1] = fn[1];
                f[2] = fn[2];
            }
            if constexpr (F32) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) two_sum_acc(hi[c][v], lo[c][v], acc[c][v]);
                    acc[c] = Acc{R(0), R(0), R(0), R(0)};
                }
            }
        }
    }

    // First half of a step on the vector units: the source's position and
    // forces from the tile, the pair's distances and far-field coefficients.
    __device__ void front(const R* tile, int j, int q, int kf, R fscale, PairPre<R>& pp, R& dx, R& dy, R& dz,
                          R* fn) const {
        const R* s = (tile + q * RW) + j * RW;  // j is uniform: no per-lane multiply
        const R sz = s[2];
        if constexpr (F32) {
            dx = (x - s[0]) + (xl - s[3]);
            dy = (y - s[1]) + (yl - s[4]);
        } else {
            dx = x - s[0];
            dy = y - s[1];
        }
        dz = z - sz;
        fn[0] = fscale * s[PW + 3 * kf];
        fn[1] = fscale * s[PW + 1 + 3 * kf];
        fn[2] = fscale * s[PW + 2 + 3 * kf];
        pp = pair_pre<R>(dx, dy, dz, z, sz);
    }

    // Second half: the overlap branch (entered by the whole wave when any lane
    // has an overlapping pair) and the written-out block.
    __device__ static PairBlock<R> back(PairPre<R>& pp, R dx, R dy, R dz) {
        if (__builtin_amdgcn_ballot_w64(pair_near(pp))) {
            __asm__ volatile("" ::: "memory");  // keep this a branch: do not speculate it
            pair_fix(pp);
        }
        return pair_block<R>(pair_fin(pp), dx, dy, dz);
    }

    // Target of accumulator entry v of this lane (offset from the first of
    // the workgroup) and its right-hand side.
    // (FP32: rows 4 (l / 16) + v of the 16 x 16 result; FP64: rows l / 16 + 4 v.)
    __device__ static int target(int v) {
        const int g = (threadIdx.x >> 4) & 3;
        return kMatWaveTargets * (threadIdx.x >> 6) + (F32 ? 4 * g + v : g + 4 * v);
    }
    __device__ static int rhs() { return threadIdx.x & 15; }
    __device__ double total(int c, int v) const {
        if constexpr (F32)
            return (double)hi[c][v] + (double)lo[c][v];
        else
            return acc[c][v];
    }
};

// Block b -> (source chunk b % splits, targets [64 (b / splits), +64)); the
// partial sums go to the same layout as pair_kernel's.
template <typename R, int K>
__global__ __launch_bounds__(kBlock) void mat_pair_kernel(const R* __restrict__ rec, int64_t N, int splits,
                                                          int64_t chunk, double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) R tile[mat_tile<R>() * rec_w<R, K>()];
    const int b = blockIdx.x;
    const int split = b % splits;
    const int64_t first = (int64_t)(b / splits) * kMatTargets;
    const int64_t s0 = (int64_t)split * chunk;
    const int64_t s1 = s0 + chunk < N ? s0 + chunk : N;
    MatLane<R, K> L;
    L.load(rec, first, N);
    L.run(rec, s0, s1, tile);
    const int k = MatLane<R, K>::rhs();
    if (k >= K) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t i = first + MatLane<R, K>::target(v);
        if (i >= N) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) part[((int64_t)(split * K + k) * 3 + c) * N + i] = L.total(c, v);
    }
}

// Batched systems on the matrix cores: as batched_kernel, with work items of
// 64 targets; five resident workgroups per CU in FP32 (the register bound
// keeps the item loop's extra registers within five waves per SIMD), four in
// FP64.
template <typename R>
constexpr int mat_batched_waves() {
    return sizeof(R) == 4 ? 5 : 4;  // FP64 spills at five
}
template <typename R, int K>
__global__ __launch_bounds__(kBlock, mat_batched_waves<R>()) void mat_batched_kernel(const R* __restrict__ rec,
                                                             const int4* __restrict__ items, int n_items,
                                                             unsigned* __restrict__ counter,
                                                             const double* __restrict__ B, double mu0, int64_t Ntot,
                                                             int kb, double* __restrict__ U) {
    __shared__ __attribute__((aligned(16))) R tile[mat_tile<R>() * rec_w<R, K>()];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        const int4 it = items[item];
        MatLane<R, K> L;
        L.load(rec, it.z, it.y);
        L.run(rec, it.x, it.y, tile);
        const int k = MatLane<R, K>::rhs();
        if (k >= kb) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = (int64_t)it.z + MatLane<R, K>::target(v);
            if (i >= it.y) continue;
            const double sc = mu0 * B[i];
#pragma unroll
            for (int c = 0; c < 3; ++c) U[((int64_t)k * Ntot + i) * 3 + c] = sc * L.total(c, v);
        }
    }
}

}  // namespace rpyw
