// Projected-axis points for pose estimation (Sec. 2.1, axis tracking).
//
// Per view: the object is segmented by a threshold on the line integrals and a
// square dilation of half-width k, and the four corner pixels of the segment
// are found.  With u the column and v the row, top-left minimises u + v,
// top-right maximises u - v (ties: smallest v), bottom-left minimises u - v,
// bottom-right maximises u + v (ties: largest v).  The dilation is not formed:
// over a dilated set, each of these keys is extreme at a window corner of a
// seed pixel (the window clipped to the detector), so every seed pixel
// contributes one candidate per corner, and the four corners are four
// integer minimum reductions of (key, tie) packed into 64 bits: exact and
// independent of the reduction order.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "cyl_internal.h"
#include "cyl_store.h"

namespace cyl {

namespace {

__device__ __forceinline__ uint64_t pack(uint32_t key, uint32_t tie) { return ((uint64_t)key << 32) | tie; }

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Saturating sum of two seed counts.
__device__ __forceinline__ uint32_t add_sat(uint32_t a, uint32_t b) { return a + b < a ? 0xffffffffu : a + b; }

// Candidates of one seed pixel (u, v): the four corners of its dilation
// window, clipped to the detector, as (key, tie) minima.
struct Corners {
    uint64_t m0, m1, m2, m3;
    uint32_t count;
    __device__ __forceinline__ void clear() {
        m0 = m1 = m2 = m3 = ~0ull;
        count = 0;
    }
    __device__ __forceinline__ void seed(int u, int v, int k, int rows, int cols) {
        const uint32_t W = (uint32_t)cols, H = (uint32_t)rows;
        const uint32_t ulo = (uint32_t)(u - k < 0 ? 0 : u - k), uhi = (uint32_t)(u + k >= cols ? cols - 1 : u + k);
        const uint32_t vlo = (uint32_t)(v - k < 0 ? 0 : v - k), vhi = (uint32_t)(v + k >= rows ? rows - 1 : v + k);
        m0 = umin64(m0, pack(ulo + vlo, vlo));                   // min u+v, smallest v
        m1 = umin64(m1, pack(W + vlo - uhi, vlo));               // max u-v, smallest v
        m2 = umin64(m2, pack(H + ulo - vhi, H - 1 - vhi));       // min u-v, largest v
        m3 = umin64(m3, pack(W + H - uhi - vhi, H - 1 - vhi));   // max u+v, largest v
        count = add_sat(count, 1u);
    }
    __device__ __forceinline__ void merge(const Corners &o) {
        m0 = umin64(m0, o.m0);
        m1 = umin64(m1, o.m1);
        m2 = umin64(m2, o.m2);
        m3 = umin64(m3, o.m3);
        count = add_sat(count, o.count);
    }
};

__device__ __forceinline__ Corners shfl_xor(const Corners &c, int o) {
    Corners r;
    r.m0 = __shfl_xor(c.m0, o);
    r.m1 = __shfl_xor(c.m1, o);
    r.m2 = __shfl_xor(c.m2, o);
    r.m3 = __shfl_xor(c.m3, o);
    r.count = __shfl_xor(c.count, o);
    return r;
}

constexpr int kCornerThreads = 1024;
constexpr int kCornerLoads = 16;  // independent loads in flight per lane

// One workgroup of 1024 lanes per view.  Lane t reads pixels t, t + 1024, ...
// kCornerLoads at a time (independent loads in flight), following (u, v) by carries
// instead of dividing.  out[view] = {TL.u, TL.v, TR.u, TR.v, BL.u, BL.v,
// BR.u, BR.v, seed count (saturated)}; corners are -1 for an empty segment.
template <int PT>
__global__ __launch_bounds__(kCornerThreads) void axis_corner_kernel(const void *__restrict__ proj, int rows, int cols,
                                                                     float threshold, int k, int32_t *__restrict__ out) {
    const int view = blockIdx.x;
    const size_t npix = (size_t)rows * cols;
    const size_t base = (size_t)view * npix;
    const uint32_t W = (uint32_t)cols, H = (uint32_t)rows;
    const int du = kCornerThreads % cols, dv = kCornerThreads / cols;
    int u = (int)threadIdx.x % cols, v = (int)threadIdx.x / cols;
    Corners c;
    c.clear();
    for (size_t j = threadIdx.x; j < npix; j += (size_t)kCornerLoads * kCornerThreads) {
        float val[kCornerLoads];
#pragma unroll
        for (int q = 0; q < kCornerLoads; ++q) {
            const size_t jq = j + (size_t)q * kCornerThreads;
            val[q] = jq < npix ? ld_any(proj, PT, base + jq) : threshold;
        }
#pragma unroll
        for (int q = 0; q < kCornerLoads; ++q) {
            if (val[q] > threshold) c.seed(u, v, k, rows, cols);
            u += du;
            const int cy = u >= cols ? 1 : 0;
            u -= cy ? cols : 0;
            v += dv + cy;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c.merge(shfl_xor(c, o));
    __shared__ Corners part[kCornerThreads / 64];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wave] = c;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kCornerThreads / 64; ++w) c.merge(part[w]);
    int32_t *o = out + (size_t)view * 9;
    const uint32_t n = c.count;
    o[8] = (int32_t)(n > 0x7fffffffu ? 0x7fffffffu : n);
    if (n == 0) {
        for (int q = 0; q < 8; ++q) o[q] = -1;
        return;
    }
    uint32_t t;
    t = (uint32_t)c.m0;
    o[0] = (int32_t)((uint32_t)(c.m0 >> 32) - t);
    o[1] = (int32_t)t;
    t = (uint32_t)c.m1;
    o[2] = (int32_t)(W + t - (uint32_t)(c.m1 >> 32));
    o[3] = (int32_t)t;
    t = H - 1 - (uint32_t)c.m2;
    o[4] = (int32_t)((uint32_t)(c.m2 >> 32) + t - H);
    o[5] = (int32_t)t;
    t = H - 1 - (uint32_t)c.m3;
    o[6] = (int32_t)(W + H - (uint32_t)(c.m3 >> 32) - t);
    o[7] = (int32_t)t;
}

// Per view: grey values left and right of the detector position centre[view]
// over rows [row_lo, row_hi]; pixel u spans [u - 1/2, u + 1/2] and is split
// at the centre in proportion.  FP64 sums in a fixed order (per-thread
// partials, then a tree), so the result does not vary between runs.
__global__ __launch_bounds__(256) void side_sum_kernel(const void *__restrict__ proj, int pt, int rows, int cols,
                                                       const double *__restrict__ centre,
                                                       const int32_t *__restrict__ row_lo,
                                                       const int32_t *__restrict__ row_hi, double *__restrict__ out) {
    const int view = blockIdx.x;
    const double c = centre[view];
    const int a = row_lo[view] < 0 ? 0 : row_lo[view];
    const int b = row_hi[view] >= rows ? rows - 1 : row_hi[view];
    const size_t base = (size_t)view * rows * cols;
    double left = 0.0, right = 0.0;
    if (a <= b) {
        const size_t n = (size_t)(b - a + 1) * cols;
        for (size_t j = threadIdx.x; j < n; j += blockDim.x) {
            const int u = (int)(j % cols);
            const double val = (double)ld_any(proj, pt, base + (size_t)a * cols + j);
            double f = c - ((double)u - 0.5);
            f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
            left += f * val;
            right += (1.0 - f) * val;
        }
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = left;
    red[1][threadIdx.x] = right;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * view] = red[0][0];
        out[2 * view + 1] = red[1][0];
    }
}

}  // namespace

}  // namespace cyl

using namespace cyl;

extern "C" int cyl_side_sums(int32_t n_views, int32_t rows, int32_t cols, const void *proj, cyl_dtype proj_type,
                             const double *centre, const int32_t *row_lo, const int32_t *row_hi, double *sums,
                             int32_t device, void *hip_stream) {
    if (n_views < 0 || rows < 1 || cols < 1 ||
        (n_views > 0 && (!proj || !centre || !row_lo || !row_hi || !sums))) {
        set_error("cyl_side_sums: need n_views >= 0, rows, cols >= 1 and non-NULL buffers");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(proj_type, "cyl_side_sums projections"))) return rc;
    if (n_views == 0) return CYL_OK;
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        set_error("cyl_side_sums: cannot select device %d", device);
        return CYL_EDEVICE;
    }
    hipLaunchKernelGGL(side_sum_kernel, dim3(n_views), dim3(256), 0, (hipStream_t)hip_stream, proj,
                       (int)proj_type, rows, cols, centre, row_lo, row_hi, sums);
    hipError_t e = hipGetLastError();
    if (prev >= 0 && prev != device) hipSetDevice(prev);
    if (e != hipSuccess) {
        set_error("cyl_side_sums: launch failed: %s", hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    return CYL_OK;
}

extern "C" int cyl_axis_corners(int32_t n_views, int32_t rows, int32_t cols, const void *proj, cyl_dtype proj_type,
                                double threshold, int32_t dilate, int32_t *corners, int32_t device,
                                void *hip_stream) {
    if (n_views < 0 || rows < 1 || cols < 1 || dilate < 0 || (n_views > 0 && (!proj || !corners))) {
        set_error("cyl_axis_corners: need n_views >= 0, rows, cols >= 1, dilate >= 0 and non-NULL buffers");
        return CYL_EINVAL;
    }
    if ((int64_t)rows + cols + 2 * (int64_t)dilate >= (1LL << 30) || (int64_t)rows * cols >= (1LL << 40)) {
        set_error("cyl_axis_corners: detector of %d x %d too large", rows, cols);
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(proj_type, "cyl_axis_corners projections"))) return rc;
    if (n_views == 0) return CYL_OK;
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        set_error("cyl_axis_corners: cannot select device %d", device);
        return CYL_EDEVICE;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    if (proj_type == CYL_F32)
        hipLaunchKernelGGL(axis_corner_kernel<CYL_F32>, dim3(n_views), dim3(kCornerThreads), 0, st, proj, rows, cols,
                           (float)threshold, dilate, corners);
    else if (proj_type == CYL_F16)
        hipLaunchKernelGGL(axis_corner_kernel<CYL_F16>, dim3(n_views), dim3(kCornerThreads), 0, st, proj, rows, cols,
                           (float)threshold, dilate, corners);
    else
        hipLaunchKernelGGL(axis_corner_kernel<CYL_BF16>, dim3(n_views), dim3(kCornerThreads), 0, st, proj, rows, cols,
                           (float)threshold, dilate, corners);
    hipError_t e = hipGetLastError();
    if (prev >= 0 && prev != device) hipSetDevice(prev);
    if (e != hipSuccess) {
        set_error("cyl_axis_corners: launch failed: %s", hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    return CYL_OK;
}
