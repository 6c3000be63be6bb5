// Device helpers shared by the fused Krylov step kernels (Lanczos and
// GMRES): fixed-order reductions, the gather of the symmetric pair kernel's
// partial sums, and loads batched ahead of their use.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sym_pairs.h"

namespace rpyw {
namespace kstep {

constexpr int kPre = 16;  // values loaded ahead of use per thread

// Sum over groups of G consecutive lanes (fixed butterfly order).
template <int G>
__device__ __forceinline__ double lane_group_sum(double s) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// out[r] = sum over c < ncol of partial[r ncol + c], r < nrows, by a
// workgroup of T threads: LPR lanes per row, lane q adding the columns
// c = q (mod LPR) in increasing order (PRE loads in flight), then an
// LPR-lane butterfly.  Ends with a barrier.
template <int T, int LPR = 8, int PRE = kPre>
__device__ void reduce_rows(const double* __restrict__ partial, int nrows, int ncol, double* out) {
    constexpr int kRows = T / LPR;
    const int rq = threadIdx.x / LPR, q = threadIdx.x % LPR;
    for (int r0 = 0; r0 < nrows; r0 += kRows) {
        const int r = r0 + rq;
        double s = 0.0;
        if (r < nrows) {
            const double* p = partial + (int64_t)r * ncol;
            for (int c = q; c < ncol; c += LPR * PRE) {
                // every load in bounds (the last column for the tail), so
                // that they issue without branches; the tail is not added
                double v[PRE];
#pragma unroll
                for (int i = 0; i < PRE; ++i) v[i] = p[c + LPR * i < ncol ? c + LPR * i : ncol - 1];
#pragma unroll
                for (int i = 0; i < PRE; ++i)
                    if (c + LPR * i < ncol) s += v[i];
            }
        }
        s = lane_group_sum<LPR>(s);
        if (q == 0 && r < nrows) out[r] = s;
    }
    __syncthreads();
}

// Entry slots of a group of n entries (3 per blob, n <= 128) whose partial
// sums a workgroup gathers: thread t takes slot t % S (S = 64, or 128 when
// n > 64) and share t / S.  Slots run over the blobs first (slot q nb + b for
// component q of blob b, nb = n / 3), so that the lanes of a wave read the
// partials of consecutive blobs, which lie next to each other.
__device__ __forceinline__ int gather_slots(int n) { return n <= 64 ? 64 : 128; }
__device__ __forceinline__ int gather_entry(int slot, int n) {
    const int nb = n / 3, q = slot / nb;
    return 3 * (slot - q * nb) + q;
}
__device__ __forceinline__ int gather_slot(int entry, int n) { return (entry % 3) * (n / 3) + entry / 3; }

// Sum of the target-chunk and source-item partials of quantity q of blob i
// (layout of sym_kernel) taken by share u of U: chunks c and items d with
// c, d = u (mod U), in increasing order, sixteen loads in flight.
template <typename R>
__device__ double gather_share(const double* __restrict__ tpart, const R* __restrict__ spart, int64_t i, int ng,
                               int C, int Hmax, int nseg, int G, int q, int u, int U) {
    const int P = (int)(i / G), t = (int)(i % G);
    const int Cs = C * nseg;
    const int nd = (sym_dmax(P, ng) + 1) * nseg;
    const int64_t st = (int64_t)3 * G;
    const double* tp = tpart + ((int64_t)P * Cs * 3 + q) * G + t;
    const R* sp = spart + ((int64_t)P * (Hmax + 1) * nseg * 3 + q) * G + t;
    double s = 0.0;
    for (int c = u; c < Cs; c += U * kPre) {
        double v[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) v[k] = c + U * k < Cs ? tp[(c + U * k) * st] : 0.0;
#pragma unroll
        for (int k = 0; k < kPre; ++k) s += v[k];
    }
    for (int d = u; d < nd; d += U * kPre) {
        double v[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) v[k] = d + U * k < nd ? (double)sp[(d + U * k) * st] : 0.0;
#pragma unroll
        for (int k = 0; k < kPre; ++k) s += v[k];
    }
    return s;
}

// A contiguous range of up to NT M values held in registers, NT threads
// taking every NT-th: load issues all of a thread's loads at once (only
// whole batches of NT that the range reaches), store writes them to LDS
// later, so that the loads overlap other work instead of each waiting for
// its value before the next is issued.
constexpr int kLdsFactor = 64 * 64;
template <int NT, int M>
struct Staged {
    double v[M];
    __device__ __forceinline__ void load(const double* __restrict__ F, int len) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i * NT >= len) break;  // uniform
            const int q = (int)threadIdx.x + i * NT;
            v[i] = F[q < len ? q : 0];
        }
    }
    __device__ __forceinline__ void store(double* Lds, int len) const {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i * NT >= len) break;
            const int q = (int)threadIdx.x + i * NT;
            if (q < len) Lds[q] = v[i];
        }
    }
};

// Sum over j < len of F[j * fs] x[j] in four partial sums (j = i (mod 4)),
// added pairwise.  The loop body has no branches, so that its LDS reads
// issue together; the last len mod 4 terms follow.
__device__ __forceinline__ double dot4(const double* __restrict__ F, int fs, const double* __restrict__ x,
                                       int len) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
#pragma unroll 2
    for (; j + 4 <= len; j += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) s4[i] = fma(F[(j + i) * fs], x[j + i], s4[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (j + i < len) s4[i] = fma(F[(j + i) * fs], x[j + i], s4[i]);
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

}  // namespace kstep
}  // namespace rpyw
