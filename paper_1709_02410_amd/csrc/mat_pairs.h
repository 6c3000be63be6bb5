// Multi-RHS products on the matrix cores (FP32C blocks of 8 or 16
// right-hand sides): the product and batched kernels that pair_kernels.hip
// launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr int kMatWaveTargets = 16;
constexpr int kMatTargets = kMatWaveTargets * (kBlock / 64);  // per workgroup
constexpr int kMatTile = 128;                                 // sources per LDS tile

template <int K>
struct MatLane {
    static constexpr int RW = rec_w<float, K>();
    float x, y, z, xl, yl;  // target l % 16 of the wave's 16
    mf4 acc[3];
    float hi[3][4], lo[3][4];

    __device__ void load(const float* __restrict__ rec, int64_t first, int64_t last) {
        int64_t i = first + kMatWaveTargets * (threadIdx.x >> 6) + (threadIdx.x & 15);
        if (i >= last) i = last - 1;
        const float* r = rec + i * RW;
        x = r[0];
        y = r[1];
        z = r[2];
        xl = r[3];
        yl = r[4];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hi[c][v] = 0.f;
                lo[c][v] = 0.f;
            }
        }
    }

    // Sum over sources [s0, s1) staged through the LDS tile.  Slots past the
    // last source of a tile, up to the next multiple of 4, hold force-free
    // blobs far from everything (their blocks are finite, their forces 0).
    __device__ void run(const float* __restrict__ rec, int64_t s0, int64_t s1, float* tile) {
        const int q = (threadIdx.x >> 4) & 3;  // source of the step
        const int k = threadIdx.x & 15;        // right-hand side
        const int kf = k < K ? k : 0;
        const float fscale = k < K ? 1.f : 0.f;
        for (int64_t t0 = s0; t0 < s1; t0 += kMatTile) {
            const int n = (int)((s1 - t0) < kMatTile ? (s1 - t0) : kMatTile);
            const int n4 = (n + 3) & ~3;
            __syncthreads();
            const float* g = rec + t0 * RW;
            for (int e = threadIdx.x; e < n * RW; e += kBlock) tile[e] = g[e];
            for (int e = n * RW + threadIdx.x; e < n4 * RW; e += kBlock) {
                const int o = e % RW;
                tile[e] = o < 2 ? 1e6f : (o == 2 ? 1.f : 0.f);
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
            PairPre<float> pp;
            float dx, dy, dz, fn[3];
            front(tile, 0, q, kf, fscale, pp, dx, dy, dz, fn);
            PairBlock<float> m = back(pp, dx, dy, dz);
            float f[3] = {fn[0], fn[1], fn[2]};
            for (int j = 0; j < n4; j += 4) {
                front(tile, j + 4 < n4 ? j + 4 : j, q, kf, fscale, pp, dx, dy, dz, fn);
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.xx, f[0], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.xy, f[0], acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.zx, f[0], acc[2], 0, 0, 0);
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.xy, f[1], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.yy, f[1], acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.zy, f[1], acc[2], 0, 0, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);  // LDS reads
                for (int i = 0; i < 6; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);  // seven VALU
                }
                const PairBlock<float> mn = back(pp, dx, dy, dz);
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.xz, f[2], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.yz, f[2], acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(m.zz, f[2], acc[2], 0, 0, 0);
                for (int i = 0; i < 3; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);
                }
                m = mn;
                f[0] = fn[0];
                f[1] = fn[1];
                f[2] = fn[2];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int v = 0; v < 4; ++v) two_sum_acc(hi[c][v], lo[c][v], acc[c][v]);
                acc[c] = mf4{0.f, 0.f, 0.f, 0.f};
            }
        }
    }

    // First half of a step on the vector units: the source's position and
    // forces from the tile, the pair's distances and far-field coefficients.
    __device__ void front(const float* tile, int j, int q, int kf, float fscale, PairPre<float>& pp, float& dx,
                          float& dy, float& dz, float* fn) const {
        const float* s = (tile + q * RW) + j * RW;  // j is uniform: no per-lane multiply
        const float sz = s[2];
        dx = (x - s[0]) + (xl - s[3]);
        dy = (y - s[1]) + (yl - s[4]);
        dz = z - sz;
        fn[0] = fscale * s[5 + 3 * kf];
        fn[1] = fscale * s[6 + 3 * kf];
        fn[2] = fscale * s[7 + 3 * kf];
        pp = pair_pre<float>(dx, dy, dz, z, sz);
    }

    // Second half: the overlap branch (entered by the whole wave when any lane
    // has an overlapping pair) and the written-out block.
    __device__ static PairBlock<float> back(PairPre<float>& pp, float dx, float dy, float dz) {
        if (__builtin_amdgcn_ballot_w64(pair_near(pp))) {
            __asm__ volatile("" ::: "memory");  // keep this a branch: do not speculate it
            pair_fix(pp);
        }
        return pair_block<float>(pair_fin(pp), dx, dy, dz);
    }

    // Target of accumulator entry v of this lane (offset from the first of
    // the workgroup) and its right-hand side.
    __device__ static int target(int v) { return kMatWaveTargets * (threadIdx.x >> 6) + 4 * ((threadIdx.x >> 4) & 3) + v; }
    __device__ static int rhs() { return threadIdx.x & 15; }
    __device__ double total(int c, int v) const { return (double)hi[c][v] + (double)lo[c][v]; }
};

// Block b -> (source chunk b % splits, targets [64 (b / splits), +64)); the
// partial sums go to the same layout as pair_kernel's.
template <int K>
__global__ __launch_bounds__(kBlock) void mat_pair_kernel(const float* __restrict__ rec, int64_t N, int splits,
                                                          int64_t chunk, double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) float tile[kMatTile * rec_w<float, K>()];
    const int b = blockIdx.x;
    const int split = b % splits;
    const int64_t first = (int64_t)(b / splits) * kMatTargets;
    const int64_t s0 = (int64_t)split * chunk;
    const int64_t s1 = s0 + chunk < N ? s0 + chunk : N;
    MatLane<K> L;
    L.load(rec, first, N);
    L.run(rec, s0, s1, tile);
    const int k = MatLane<K>::rhs();
    if (k >= K) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t i = first + MatLane<K>::target(v);
        if (i >= N) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) part[((int64_t)(split * K + k) * 3 + c) * N + i] = L.total(c, v);
    }
}

// Batched systems on the matrix cores: as batched_kernel, with work items of
// 64 targets; five resident workgroups per CU (the register bound keeps the
// item loop's extra registers within five waves per SIMD).
constexpr int kMatBatchedWaves = 5;
template <int K>
__global__ __launch_bounds__(kBlock, kMatBatchedWaves) void mat_batched_kernel(const float* __restrict__ rec,
                                                             const int4* __restrict__ items, int n_items,
                                                             unsigned* __restrict__ counter,
                                                             const double* __restrict__ B, double mu0, int64_t Ntot,
                                                             int kb, double* __restrict__ U) {
    __shared__ __attribute__((aligned(16))) float tile[kMatTile * rec_w<float, K>()];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        const int4 it = items[item];
        MatLane<K> L;
        L.load(rec, it.z, it.y);
        L.run(rec, it.x, it.y, tile);
        const int k = MatLane<K>::rhs();
        if (k >= kb) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = (int64_t)it.z + MatLane<K>::target(v);
            if (i >= it.y) continue;
            const double sc = mu0 * B[i];
#pragma unroll
            for (int c = 0; c < 3; ++c) U[((int64_t)k * Ntot + i) * 3 + c] = sc * L.total(c, v);
        }
    }
}

}  // namespace rpyw
