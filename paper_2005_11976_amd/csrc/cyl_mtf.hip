// Directional MTF of a reconstructed volume (Sec. 2.3, Eq. 8).
//
// The measurement runs on the central h-slice (the middle slice, or the mean
// of the two middle slices for an even number of slices) in FP64.  Each
// output is the modulation m = (max - min) / (max + min) of a set of cells of
// that slice: one ring (the azimuthal MTF at that radius) or the rings of one
// window of `window` rings, windows slid by their own width (the radial MTF's
// radial dependence).  Max and min are exact in any order and the ratio is
// one correctly rounded FP64 division, so the result does not depend on the
// reduction order.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "cyl_internal.h"
#include "cyl_store.h"

namespace cyl {

namespace {

// One workgroup per output.  window = 0: output r covers ring r (all theta);
// window = w: output k covers rings [k w, (k + 1) w).
__global__ __launch_bounds__(256) void mtf_kernel(const void *__restrict__ vol, int vt, int n_h, int n_theta,
                                                  int n_r, int window, double *__restrict__ out) {
    const int o = blockIdx.x;
    const size_t plane = (size_t)n_theta * n_r;
    const size_t s0 = (size_t)((n_h - 1) / 2) * plane, s1 = (size_t)(n_h / 2) * plane;
    const bool two = (n_h % 2) == 0;
    const int r0 = window == 0 ? o : o * window;
    const int nw = window == 0 ? 1 : window;
    const int n = n_theta * nw;
    double hi = -INFINITY, lo = INFINITY;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int t = j / nw, r = r0 + j % nw;
        const size_t c = (size_t)t * n_r + r;
        double x = (double)ld_any(vol, vt, s0 + c);
        if (two) x = 0.5 * (x + (double)ld_any(vol, vt, s1 + c));
        hi = fmax(hi, x);
        lo = fmin(lo, x);
    }
    __shared__ double rh[256], rl[256];
    rh[threadIdx.x] = hi;
    rl[threadIdx.x] = lo;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            rh[threadIdx.x] = fmax(rh[threadIdx.x], rh[threadIdx.x + s]);
            rl[threadIdx.x] = fmin(rl[threadIdx.x], rl[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double a = rh[0], b = rl[0];
        out[o] = (a + b == 0.0) ? 0.0 : (a - b) / (a + b);
    }
}

}  // namespace

}  // namespace cyl

using namespace cyl;

extern "C" int cyl_mtf(int32_t n_h, int32_t n_theta, int32_t n_r, const void *vol, cyl_dtype vol_type,
                       int32_t window, double *out, int32_t device, void *hip_stream) {
    if (n_h < 1 || n_theta < 1 || n_r < 1 || window < 0 || window > n_r || !vol || !out) {
        set_error("cyl_mtf: need n_h, n_theta, n_r >= 1, 0 <= window <= n_r and non-NULL buffers");
        return CYL_EINVAL;
    }
    if ((int64_t)n_theta * (window == 0 ? 1 : window) >= (1LL << 31)) {
        set_error("cyl_mtf: %d x %d cells per output is too many", n_theta, window);
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vol_type, "cyl_mtf volume"))) return rc;
    const int n_out = window == 0 ? n_r : n_r / window;
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        set_error("cyl_mtf: cannot select device %d", device);
        return CYL_EDEVICE;
    }
    hipLaunchKernelGGL(mtf_kernel, dim3(n_out), dim3(256), 0, (hipStream_t)hip_stream, vol, (int)vol_type, n_h,
                       n_theta, n_r, window, out);
    hipError_t e = hipGetLastError();
    if (prev >= 0 && prev != device) hipSetDevice(prev);
    if (e != hipSuccess) {
        set_error("cyl_mtf: launch failed: %s", hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    return CYL_OK;
}
