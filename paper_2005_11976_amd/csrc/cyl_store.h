// Storage types of volumes, projections and weights, shared by every kernel
// file: FP32, FP16 and BF16 values are widened to FP32 on load and rounded to
// nearest-even on store (the FP16/BF16 storage of the mixed-precision runs;
// all arithmetic is FP32 or wider).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/cyl.h"

namespace cyl {

__device__ __forceinline__ float bf16_to_f32(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }

// Nearest-even rounding of an FP32 value to BF16 (NaNs stay quiet NaNs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int DT>
struct Store;
// ld/st: plain global access.  ldb: load element i through a buffer resource
// (32-bit offsets, range-checked by the hardware: an offset past the end reads
// 0), used for the gathers of the traversal.
template <>
struct Store<CYL_F32> {
    static constexpr int kSize = 4;
    static __device__ __forceinline__ float ld(const void *p, size_t i) { return ((const float *)p)[i]; }
    static __device__ __forceinline__ void st(void *p, size_t i, float v) { ((float *)p)[i] = v; }
    static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t rs, unsigned i) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, i << 2, 0, 0));
    }
};
template <>
struct Store<CYL_F16> {
    static constexpr int kSize = 2;
    static __device__ __forceinline__ float ld(const void *p, size_t i) {
        return __half2float(((const __half *)p)[i]);
    }
    static __device__ __forceinline__ void st(void *p, size_t i, float v) {
        ((__half *)p)[i] = __float2half_rn(v);
    }
    static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t rs, unsigned i) {
        const unsigned short x = __builtin_amdgcn_raw_buffer_load_b16(rs, i << 1, 0, 0);
        return __half2float(__builtin_bit_cast(__half, x));
    }
};
template <>
struct Store<CYL_BF16> {
    static constexpr int kSize = 2;
    static __device__ __forceinline__ float ld(const void *p, size_t i) {
        return bf16_to_f32(((const uint16_t *)p)[i]);
    }
    static __device__ __forceinline__ void st(void *p, size_t i, float v) {
        ((uint16_t *)p)[i] = f32_to_bf16(v);
    }
    static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t rs, unsigned i) {
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(rs, i << 1, 0, 0));
    }
};

// Buffer resource over n bytes at p (gfx9 word 3: 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)nbytes, 0x00020000);
}

// Load / store of an array whose storage type is a runtime value (weights,
// the comparison kernels); the switch is uniform across the wave.
__device__ __forceinline__ float ld_any(const void *p, int dt, size_t i) {
    if (dt == CYL_F32) return Store<CYL_F32>::ld(p, i);
    if (dt == CYL_F16) return Store<CYL_F16>::ld(p, i);
    return Store<CYL_BF16>::ld(p, i);
}
__device__ __forceinline__ void st_any(void *p, int dt, size_t i, float v) {
    if (dt == CYL_F32)
        Store<CYL_F32>::st(p, i, v);
    else if (dt == CYL_F16)
        Store<CYL_F16>::st(p, i, v);
    else
        Store<CYL_BF16>::st(p, i, v);
}

}  // namespace cyl
