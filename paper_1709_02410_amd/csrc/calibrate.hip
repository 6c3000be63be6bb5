// Instrumentation: kernels with an exactly known count of vector-ALU
// instructions, against which hardware counters (instruction and FLOP
// counts) are calibrated before they are used to report the FLOP rate of
// the pair kernels.
//
// kind 0: FP32 fused multiply-adds, kind 1: FP64 fused multiply-adds.  Each
// wave runs `iters` iterations of 8 independent chains x <- x * b + c with
// b, c in vector registers: exactly 8 * iters FMA instructions per wave
// (64 lanes, 2 FLOP each), plus a loop counter and a final store.
#include "pair_math.h"
#include "rpyw_internal.h"

namespace rpyw {

namespace {

template <typename R>
__global__ __launch_bounds__(256) void calib_fma_kernel(int iters, R b, R c, R* __restrict__ out) {
    const R bb = b + (R)threadIdx.x * (R)1e-9, cc = c - (R)threadIdx.x * (R)1e-9;
    R x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (R)(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fma_(x[k], bb, cc);
    }
    R s = x[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) s += x[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

}  // namespace rpyw

using namespace rpyw;

extern "C" int rpy_wall_calibrate(int kind, int64_t blocks, int32_t iters, void* out, void* stream) {
    if ((kind != 0 && kind != 1) || blocks < 1 || blocks > (1 << 20) || iters < 1 || !out) return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0)
        hipLaunchKernelGGL(calib_fma_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0000001f,
                           0.9999999f, (float*)out);
    else
        hipLaunchKernelGGL(calib_fma_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0000000001,
                           0.9999999999, (double*)out);
    RPYW_HIP(hipGetLastError());
    return RPYW_OK;
}
