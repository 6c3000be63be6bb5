// Per-blob records consumed by the pair kernels: scaled, regularised
// position (x/a, y/a, max(z, a)/a), FP32 low parts of x and y in the FP32
// layout, then B f for each right-hand side (B = min(z/a, 1), the blob-wall
// regularisation factor), zero-padded to a 16-byte multiple.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rpyw {

template <typename R>
constexpr int pos_slots() {
    return sizeof(R) == 4 ? 5 : 3;
}
template <typename R, int K>
constexpr int rec_w() {
    return sizeof(R) == 4 ? (5 + 3 * K + 3) / 4 * 4 : (3 + 3 * K + 1) / 2 * 2;
}

// The record of blob i (i < N) into r[0 .. recw): RHS k is read from
// F + k N 3 ([kb][N][3]); when F2 is given (kb = 2) the second RHS is read
// from F2 instead.  With a periodic cell (lx, ly > 0, units of a) x and y
// are wrapped into [0, lx) and [0, ly) first, in FP64, so that differences
// stay below one cell length.  Blobs i >= N are padding: force-free blobs
// far from everything (x = y = 1e6 a, B = 0).  *B receives the blob's B.
template <typename R>
__device__ __forceinline__ void make_record(const double* __restrict__ pos, const double* __restrict__ F, int64_t N,
                                            int kb, int recw, double inv_a, const double* __restrict__ F2, double lx,
                                            double ly, int64_t i, R* r, double* B) {
    if (i >= N) {
        for (int e = 0; e < recw; ++e) r[e] = R(0);
        r[0] = R(1e6);
        r[1] = R(1e6);
        r[2] = R(1);
        *B = 0.0;
        return;
    }
    double x = pos[3 * i] * inv_a, y = pos[3 * i + 1] * inv_a;
    const double z = pos[3 * i + 2] * inv_a;
    if (lx > 0.0) {
        x -= lx * floor(x / lx);
        y -= ly * floor(y / ly);
    }
    const double b = z < 1.0 ? z : 1.0;
    const double zt = z < 1.0 ? 1.0 : z;
    int o;
    if constexpr (sizeof(R) == 4) {
        const float xh = (float)x, yh = (float)y;
        r[0] = xh;
        r[1] = yh;
        r[2] = (float)zt;
        r[3] = (float)(x - (double)xh);
        r[4] = (float)(y - (double)yh);
        o = 5;
    } else {
        r[0] = x;
        r[1] = y;
        r[2] = zt;
        o = 3;
    }
    for (int k = 0; k < kb; ++k) {
        const double* src = (F2 && k == 1) ? F2 + i * 3 : F + (k * N + i) * 3;
        for (int c = 0; c < 3; ++c) r[o + 3 * k + c] = (R)(b * src[c]);
    }
    for (int e = o + 3 * kb; e < recw; ++e) r[e] = R(0);
    *B = b;
}

// Records for blobs [0, Npad) (make_record; Npad >= N), and B when Bout is
// given.
template <typename R>
__global__ void pack_kernel(const double* __restrict__ pos, const double* __restrict__ F, int64_t N, int kb,
                            int recw, double inv_a, R* __restrict__ rec, double* __restrict__ Bout,
                            const double* __restrict__ F2, double lx, double ly, int64_t Npad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Npad) return;
    double b;
    make_record<R>(pos, F, N, kb, recw, inv_a, F2, lx, ly, i, rec + i * recw, &b);
    if (Bout) Bout[i] = b;
}

}  // namespace rpyw
