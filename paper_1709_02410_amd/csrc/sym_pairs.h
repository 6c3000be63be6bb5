// Symmetric evaluation of pair sums: every unordered pair (i, j) is
// evaluated once and contributes to both blobs.  This uses the reciprocity
// of the blob mobility (M_ji = M_ij^T, arXiv:1709.02410 Sec. II.A: M is
// symmetric), under which the transposed block is the same coefficient set
// with the two off-diagonal wall coefficients exchanged.
//
// Work decomposition.  Blobs are grouped by G = 64 NB (NB 64-lane blocks:
// NB = 4 for large problems, NB = 1 when there would be too few groups to
// fill the GPU).  Work item (P, d) pairs target group P with source group
// Q = (P + d) mod ng for d = 0 .. H(P) (sym_rowlen), which covers every
// unordered pair of groups exactly once.  A workgroup of NB waves takes
// `ipw` consecutive items of one row.  Wave w holds target block NB P + w;
// in phase b (b = 0 .. NB-1) it takes source block (w + b) mod NB, so the
// waves work on different source blocks (in FP64 with a workgroup barrier
// between phases).  A phase is 64
// steps in which lane l pairs its target with source (l + s) mod 64, read
// from LDS rows that hold the block twice (so l + s needs no wrap).  The lane
// adds the target-side contribution to its own sums.  The source-side
// contribution goes, in FP32, to an accumulator that moves one lane down
// after every step (a DPP wavefront rotate fused into the add), so that
// after the phase lane l holds the complete sum of source l, and the
// waves' sums are added through LDS; in FP64 it goes to an LDS slot l + s of
// that source block by an LDS atomic add (no two lanes of an instruction
// share a slot, one wave owns a block per phase and the phases are ordered
// by the barriers, so the order of additions is fixed; slots j and j + 64
// together hold source j's sum).
// In the diagonal item (d = 0) blocks above the wave's own are done
// symmetrically, the wave's own block over all ordered pairs (self
// included, target side only), and blocks below it are left to the waves
// that own them.  When there are few items, every item's passes are split
// into nseg segments of 64 / nseg steps, each its own workgroup.  Target
// sums are written per (row, chunk, segment) and source sums per (group, d,
// segment); an epilogue adds both in a fixed order, so results are bitwise
// reproducible.
//
// A Body supplies the per-pair arithmetic: KREC right-hand sides in the
// record, NQ accumulated quantities, the unroll factor of the 64-step loop,
// and
//   template <bool SYM> static void pair(const SymTarget&, const R* rec,
//                                        R (&acc)[NQ], R (&src)[NQ],
//                                        const Box<R>&);
// which adds the target-side contribution to acc and, when SYM, writes the
// source-side contribution to src.  A Body with kDuo set also supplies
//   template <bool SYM> static void pair2(const SymTarget&, const R* ra,
//                                         const R* rb, R (&acc)[NQ],
//                                         R (&sa)[NQ], R (&sb)[NQ]);
// for two consecutive sources at once (the 64-step loop then takes two
// steps per iteration).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pair_math.h"
#include "records.h"

namespace rpyw {

// Pseudo-periodic cell along the wall, units of a: lengths, the lengths
// split into a high part with 12 significant bits (small integer multiples
// of it are exact) plus the rest, and the inverse lengths.  Unused by bodies
// for the open domain.
template <typename R>
struct Box {
    R lx, ly, lxh, lxl, lyh, lyl, ilx, ily;
};

// Number of source-group offsets d > 0 that row P owns (ng groups).
__host__ __device__ inline int sym_rowlen(int P, int ng) {
    return (ng & 1) ? (ng - 1) / 2 : ng / 2 - 1 + (P < ng / 2 ? 1 : 0);
}

// Last source slot d of group P that some item fills (see sym_rowlen).
__host__ __device__ inline int sym_dmax(int P, int ng) {
    const int hmax = ng / 2;
    return ((ng & 1) == 0 && P < ng / 2) ? hmax - 1 : hmax;
}

// Lane l receives the value held by lane (l + 1) mod 64.
__device__ __forceinline__ float rot_next(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double rot_next(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x134, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// rot_next(s) + c.  The rotation takes c as its old value (never read: the
// rotate has a source lane for every lane, and bound_ctrl is set), which
// keeps it next to the add that consumes it, so the two fuse into one DPP
// add instead of a DPP move and an add.
__device__ __forceinline__ float rot_add(float s, float c) {
    const int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, c), __builtin_bit_cast(int, s), 0x134, 0xF, 0xF,
                                              true);
    return __builtin_bit_cast(float, r) + c;
}
__device__ __forceinline__ double rot_add(double s, double c) { return rot_next(s) + c; }

template <typename R>
struct Vec;
template <>
struct Vec<float> {
    using T = float4;
    static constexpr int W = 4;
    __device__ static float get(const float4& v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }
    __device__ static float4 make(const float* p) { return make_float4(p[0], p[1], p[2], p[3]); }
};
template <>
struct Vec<double> {
    using T = double2;
    static constexpr int W = 2;
    __device__ static double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static double2 make(const double* p) { return make_double2(p[0], p[1]); }
};

// Inputs of the records when the kernel forms them itself (make_record):
// positions [N][3], kb right-hand sides [kb][N][3], 1 / a and the periodic
// cell in units of a (zeros for the open domain).
struct PackSrc {
    const double* pos;
    const double* F;
    int64_t N;
    int kb;
    double inv_a, lx, ly;
};

// The target a lane holds: scaled position (FP32: plus low parts) and the
// record's right-hand sides.
template <typename R, int KREC>
struct SymTarget {
    R x, y, z, xl, yl;
    R f[KREC][3];
};

// Difference vector target - source of a record (FP32: hi/lo parts).
template <typename R, int KREC>
__device__ __forceinline__ void sym_diff(const SymTarget<R, KREC>& t, const R* r, R& dx, R& dy, R& dz) {
    dx = t.x - r[0];
    dy = t.y - r[1];
    if constexpr (sizeof(R) == 4) {
        dx += t.xl - r[3];
        dy += t.yl - r[4];
    }
    dz = t.z - r[2];
}

template <typename R, class Body>
struct SymLane {
    static constexpr int KREC = Body::KREC;
    static constexpr int NQ = Body::NQ;
    static constexpr int RW = rec_w<R, KREC>();
    static constexpr int NV = RW / Vec<R>::W;
    SymTarget<R, KREC> t;
    R acc[NQ], hi[NQ], lo[NQ];

    __device__ void load(const R* __restrict__ r) {
        t.x = r[0];
        t.y = r[1];
        t.z = r[2];
        t.xl = sizeof(R) == 4 ? r[3] : R(0);
        t.yl = sizeof(R) == 4 ? r[4] : R(0);
#pragma unroll
        for (int k = 0; k < KREC; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) t.f[k][c] = r[pos_slots<R>() + 3 * k + c];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = hi[q] = lo[q] = R(0);
    }

    // One 64-step pass over source block `blk`.  When SYM, the source-side
    // contribution for source (l + s) mod 64 goes either to the accumulator
    // S, which moves one lane down after every step (a DPP wave rotate fused
    // into the add), so that after the pass lane l holds source l's sum
    // (FP32; sa is null), or to LDS sa[q * 128 + l + s] by an atomic add
    // (FP64).
    // vs: LDS entries per vector slot of the tile (128 per source block).
    // Steps s0 .. s1 - 1 only (a segment of the pass; s1 - s0 even): the
    // rotating accumulator then ends with source (l + s1) mod 64 in lane l.
    template <bool SYM>
    __device__ void pass(const typename Vec<R>::T* __restrict__ tile, int vs, int blk, int l, R* sa, R (&S)[NQ],
                         const Box<R>& box, int s0 = 0, int s1 = 64) {
        using VT = typename Vec<R>::T;
        const VT* base = tile + blk * 128 + l;
        R* sl = sa + l;
#pragma unroll
        for (int q = 0; q < NQ; ++q) S[q] = R(0);
        // Source side of step s: to the LDS slots (FP64, sa given) or into
        // the rotating accumulator (FP32, sa null); chosen at compile time.
        auto source_side = [&](const R(&c)[NQ], int s) {
            if constexpr (sizeof(R) == 8) {
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    __hip_atomic_fetch_add(sl + q * 128 + s, c[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    S[q] = rot_add(S[q], c[q]);
                    // An empty asm use pins the add to this pair's block:
                    // otherwise the tail of the pair is sunk past the next
                    // overlap branch, away from the (unmovable) DPP rotate it
                    // should fuse with.
                    __asm__ volatile("" ::"v"(S[q]));
                }
            }
        };
        auto fetch = [&](R(&r)[RW], int s) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const VT q = base[v * vs + s];
#pragma unroll
                for (int e = 0; e < Vec<R>::W; ++e) r[v * Vec<R>::W + e] = Vec<R>::get(q, e);
            }
        };
        if constexpr (Body::kDuo) {
            // Two steps per iteration sharing one overlap branch; not
            // unrolled further (fewer registers, and more waves per SIMD).
#pragma unroll 1
            for (int s = s0; s < s1; s += 2) {
                R ra[RW], rb[RW], ca[NQ], cb[NQ];
                fetch(ra, s);
                fetch(rb, s + 1);
                Body::template pair2<SYM>(t, ra, rb, acc, ca, cb);
                if constexpr (SYM) {
                    source_side(ca, s);
                    source_side(cb, s + 1);
                }
            }
        } else {
#pragma unroll Body::kUnroll
            for (int s = s0; s < s1; ++s) {
                R r[RW], c[NQ];
                fetch(r, s);
                Body::template pair<SYM>(t, r, acc, c, box);
                if constexpr (SYM) source_side(c, s);
            }
        }
        if constexpr (SYM) {
            if (!sa) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) S[q] = rot_next(S[q]);
            }
        }
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                two_sum_acc(hi[q], lo[q], acc[q]);
                acc[q] = R(0);
            }
        }
    }

    __device__ double total(int q) const {
        if constexpr (sizeof(R) == 4)
            return (double)hi[q] + (double)lo[q];
        else
            return (double)acc[q];
    }
};

// Groups of G = 64 NB blobs (NB blocks of 64, one wave each): NB = 4 for
// large problems, NB = 1 to have enough workgroups when there are few groups.
// Small problems split every item's 64-step passes into segments: NS
// segments are NS waves of one workgroup (NB = 1), which hold the same
// target block, take 64 / NS consecutive steps each and add their sums
// through LDS in wave order; beyond that, nseg segments are workgroups of
// their own (nseg = 1, 2 or 4), each writing its own partials.
// rec: ng * G records (padded with force-free blobs far away), or, with FP,
// none: every workgroup forms the records of its target and source groups
// from ps (make_record) as it loads them, which saves small problems the
// launch of the packing kernel.
// tpart: [ng * C * nseg][NQ][G] doubles; spart: [ng * (Hmax + 1) * nseg][NQ][G].
template <typename R, class Body, int NB = 4, int NS = 1, bool FP = false>
__global__ __launch_bounds__(64 * NB * NS) void sym_kernel(const R* __restrict__ rec, int ng, int C, int ipw,
                                                           int Hmax, int nseg, double* __restrict__ tpart,
                                                           R* __restrict__ spart, Box<R> box, PackSrc ps) {
    static_assert(NS == 1 || NB == 1, "step segments within a workgroup need one target block");
    using L = SymLane<R, Body>;
    using VT = typename Vec<R>::T;
    constexpr int NQ = L::NQ;
    constexpr int G = 64 * NB;
    constexpr int NW = NB * NS;   // waves
    constexpr int VS = 128 * NB;  // tile entries per vector slot
    // FP64: source sums by LDS atomics (one wave per source block and phase);
    // FP32: by the DPP rotation, then across the waves through `red` (LDS
    // FP32 atomic adds are far slower than the rotation on this GPU, FP64
    // ones are faster).
    constexpr bool kLds = sizeof(R) == 8;
    __shared__ VT tile[L::NV * VS];
    // per source block (NS = 1) or per step segment (NS > 1), slots l + s
    __shared__ R sacc[kLds ? NW : 1][kLds ? NQ : 1][kLds ? 128 : 1];
    __shared__ double tred[NS > 1 ? NS : 1][NS > 1 ? NQ : 1][NS > 1 ? 64 : 1];  // target sums of the step segments
    // FP32 with more than three quantities per blob (the VJP, several
    // right-hand sides): the NB phases' passes are added into one row of G
    // slots per quantity in phase order, with a barrier between phases, which
    // needs NB times less LDS and so allows more workgroups per CU.  With
    // three (the product) the waves write separate rows and one barrier
    // follows the last phase (fewer barriers, and occupancy is bounded by
    // registers there).
    constexpr bool kPhased = !kLds && NQ > 3 && NS == 1;
    __shared__ R red[kLds ? 1 : (kPhased ? 1 : NW)][kLds ? 1 : NQ][kLds ? 1 : G];
    const int g = blockIdx.x % nseg, P = blockIdx.x / nseg / C, c = blockIdx.x / nseg % C;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int w = NS > 1 ? 0 : wave;     // target block of the wave
    const int seg = NS > 1 ? wave : 0;   // step segment of the wave
    const int s0 = (g * NS + seg) * (64 / (nseg * NS)), s1 = s0 + 64 / (nseg * NS);
    const bool loader = NS == 1 || threadIdx.x < G;  // one thread per record of a group
    L me;
    if constexpr (FP) {
        R rr[L::RW];
        double bd;
        make_record<R>(ps.pos, ps.F, ps.N, ps.kb, L::RW, ps.inv_a, nullptr, ps.lx, ps.ly, (int64_t)P * G + w * 64 + l,
                       rr, &bd);
        me.load(rr);
    } else {
        me.load(rec + ((int64_t)P * G + w * 64 + l) * L::RW);
    }
    const int H = sym_rowlen(P, ng);
    const int d0 = c * ipw;
    const int d1 = d0 + ipw - 1 < H ? d0 + ipw - 1 : H;
    for (int d = d0; d <= d1; ++d) {
        const int Q = (P + d) % ng;
        __syncthreads();
        {
            const int b = threadIdx.x >> 6, j = threadIdx.x & 63;
            if (loader) {
                if constexpr (FP) {
                    R rr[L::RW];
                    double bd;
                    make_record<R>(ps.pos, ps.F, ps.N, ps.kb, L::RW, ps.inv_a, nullptr, ps.lx, ps.ly,
                                   (int64_t)Q * G + threadIdx.x, rr, &bd);
#pragma unroll
                    for (int v = 0; v < L::NV; ++v) {
                        const VT q = Vec<R>::make(rr + v * Vec<R>::W);
                        tile[v * VS + b * 128 + j] = q;
                        tile[v * VS + b * 128 + j + 64] = q;
                    }
                } else {
                    const VT* gr = reinterpret_cast<const VT*>(rec + ((int64_t)Q * G + threadIdx.x) * L::RW);
#pragma unroll
                    for (int v = 0; v < L::NV; ++v) {
                        const VT q = gr[v];
                        tile[v * VS + b * 128 + j] = q;
                        tile[v * VS + b * 128 + j + 64] = q;
                    }
                }
            }
            if constexpr (kLds) {
                R* z = &sacc[0][0][0];
                for (int e = threadIdx.x; e < NW * NQ * 128; e += blockDim.x) z[e] = R(0);
            }
        }
        __syncthreads();
        for (int bb = 0; bb < NB; ++bb) {
            const int blk = (w + bb) % NB;
            R S[NQ];
            if (d == 0 && blk < w) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) S[q] = R(0);
            } else if (d == 0 && blk == w) {
                me.template pass<false>(tile, VS, blk, l, nullptr, S, box, s0, s1);
            } else {
                me.template pass<true>(tile, VS, blk, l, kLds ? &sacc[NS > 1 ? seg : blk][0][0] : nullptr, S, box,
                                       s0, s1);
            }
            if constexpr (kPhased) {
                R* slot = &red[0][0][blk * 64 + ((l + s1) & 63)];
#pragma unroll
                for (int q = 0; q < NQ; ++q) slot[q * G] = bb == 0 ? S[q] : slot[q * G] + S[q];
            } else if constexpr (!kLds) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) red[wave][q][blk * 64 + ((l + s1) & 63)] = S[q];
            }
            if constexpr (kLds || kPhased) __syncthreads();  // one wave per source block in every phase
        }
        if constexpr (!kLds && !kPhased) __syncthreads();
        R* out = spart + (((int64_t)Q * (Hmax + 1) + d) * nseg + g) * NQ * G;
        const int b = threadIdx.x >> 6, j = threadIdx.x & 63;
        if (loader) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if constexpr (kLds && NS > 1) {
                    R t = sacc[0][q][j] + sacc[0][q][j + 64];
#pragma unroll
                    for (int k = 1; k < NS; ++k) t += sacc[k][q][j] + sacc[k][q][j + 64];
                    out[q * G + threadIdx.x] = t;
                } else if constexpr (kLds) {
                    out[q * G + threadIdx.x] = sacc[b][q][j] + sacc[b][q][j + 64];
                } else if constexpr (kPhased) {
                    out[q * G + threadIdx.x] = red[0][q][threadIdx.x];
                } else {
                    R t = red[0][q][threadIdx.x];
#pragma unroll
                    for (int k = 1; k < NW; ++k) t += red[k][q][threadIdx.x];
                    out[q * G + threadIdx.x] = t;
                }
            }
        }
    }
    double* tp = tpart + (int64_t)blockIdx.x * NQ * G;  // chunk c * nseg + g of row P
    if constexpr (NS > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tred[seg][q][l] = me.total(q);
        __syncthreads();
        if (threadIdx.x < G) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double t = tred[0][q][l];
#pragma unroll
                for (int k = 1; k < NS; ++k) t += tred[k][q][l];
                tp[q * G + threadIdx.x] = t;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) tp[q * G + threadIdx.x] = me.total(q);
    }
}

// Part u of U of the sum of quantity q of blob i over the chunk target
// partials and the item source partials (nseg of each per chunk and item):
// chunks c and items d with c, d = u (mod U), in a fixed order.  U = 1 gives
// the whole sum.
template <typename R>
__device__ __forceinline__ double sym_gather(const double* __restrict__ tpart, const R* __restrict__ spart, int64_t i,
                                             int ng, int C, int Hmax, int NQ, int q, int G = 256, int u = 0,
                                             int U = 1, int nseg = 1) {
    const int P = (int)(i / G), t = (int)(i % G);
    const int Cs = C * nseg;
    const int dmax = (sym_dmax(P, ng) + 1) * nseg - 1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const double* tp = tpart + ((int64_t)P * Cs * NQ + q) * G + t;
    const int64_t tst = (int64_t)NQ * G;
    int c = u;
    for (; c + U < Cs; c += 2 * U) {
        s2 += tp[c * tst];
        s3 += tp[(c + U) * tst];
    }
    if (c < Cs) s2 += tp[c * tst];
    const R* sp = spart + ((int64_t)P * (Hmax + 1) * nseg * NQ + q) * G + t;
    const int64_t st = tst;
    int d = u;
    for (; d + 3 * U <= dmax; d += 4 * U) {
        s0 += (double)sp[d * st];
        s1 += (double)sp[(d + U) * st];
        s2 += (double)sp[(d + 2 * U) * st];
        s3 += (double)sp[(d + 3 * U) * st];
    }
    for (; d <= dmax; d += U) s0 += (double)sp[d * st];
    return (s0 + s1) + (s2 + s3);
}

}  // namespace rpyw
