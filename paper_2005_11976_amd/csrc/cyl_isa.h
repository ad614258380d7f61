// Single-instruction ALU helpers of the traversal kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace cyl {

// Reciprocal, square root and reciprocal square root: the hardware
// approximations (about 1 ulp), without the IEEE fix-up sequences.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// min / max of loop-carried values without the canonicalising moves the
// compiler otherwise inserts before every v_min/v_max (the operands are never
// signalling NaNs: they come from arithmetic or are +inf)
__device__ __forceinline__ float vmin3(float a, float b, float c) {
    float d;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}
__device__ __forceinline__ float vmin(float a, float b) {
    float d;
    asm("v_min_f32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
}
__device__ __forceinline__ float vmax(float a, float b) {
    float d;
    asm("v_max_f32 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

// floor(x + 1/2) as an integer in one instruction (round to nearest, ties
// upward): the fixed-point sums need a fixed rounding rule, not a particular one.
__device__ __forceinline__ int round_half_up(float x) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// 24-bit integer multiply-add (cell indices are below 2^24 by construction).
__device__ __forceinline__ unsigned mul24(int a, int b) { return __umul24(a, b); }

}  // namespace cyl
