/* Host stand-in for <hip/hip_runtime.h>: lets the device pair arithmetic
 * (paper_1709_02410_amd/csrc/pair_math.h) compile with g++ for CPU tests. */
#pragma once
#include <cmath>
#define __device__
#define __forceinline__ inline
#define __builtin_amdgcn_rsqf(x) (1.0f / std::sqrt((float)(x)))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt((double)(x)))
#define __builtin_amdgcn_ballot_w64(b) ((unsigned long long)(b))
