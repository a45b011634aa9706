// Device-side helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace vp {

// tanh(x) = sign(x) (1 - e) / (1 + e) with e = exp(-2|x|) = 2^(-2 log2(e) |x|).
// Uses the hardware exp2 and reciprocal (about 1 ulp each): absolute error a few
// units of 2^-24, which is what FP32 storage of activations of size <= 1 costs
// anyway.  Saturates to +-1 for large |x| (exp2 underflows to 0) and keeps NaN.
__device__ __forceinline__ float tanh_f32(float x) {
    const float ax = __builtin_fabsf(x);
    const float e = __builtin_amdgcn_exp2f(ax * -2.8853900817779268f);
    const float r = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    return __builtin_copysignf(r, x);
}

// sum over the 64 lanes of a wavefront (every lane receives the total)
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace vp
