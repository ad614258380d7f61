// The paper's own projector pair (Sec. 2.2), kept beside the exact pair as a
// comparison of cost and accuracy.
//
// Forward projection, pixel driven: the ray from the source to the pixel
// centre is sampled at distances d_k = (k + 1/2) step from the source
// (d_k < the pixel's distance); every sample inside the grid support goes
// through the cylindrical transform (Eq. 2) and adds step * mu there, mu
// taken from the cell holding the sample (nearest: t_jl = step x samples in
// cell l) or interpolated trilinearly between cell centres in (r, theta, h)
// (theta periodic, r and h clamped to the first and last centres).  Its row
// sum is step x (samples in the support).
//
// Back-projection, voxel driven: each cell centre is projected into the view
// and the image is read there bilinearly between pixel centres (pixels off the
// detector read nothing); the bilinear weights summed over the views are the
// cell's column normalisation.  It is not the transpose of the forward
// projection.  Both run in FP32 (the projection of a cell centre through the
// view's FP32 inverse detector matrix).

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "cyl_internal.h"
#include "cyl_store.h"

namespace cyl {

namespace {

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Samples kb, kb + 1, ..., kb + n - 1 of the ray a + d e (|e| = 1,
// d in (0, len)), d_k = (k + 1/2) step, that cover the part inside the
// cylinder r <= r_max and the slab h_min <= h <= h_max (FP64), with one sample
// of margin either side; the samples are then tested one by one.  kb is a
// double (the source may be far away), n at most the support diameter / step
// + 4 (bounded on the host).
__device__ bool sample_range(const GeomDev &g, const double *a, const double *e, double len, double step, double &kb,
                             int &n) {
    double lo = 0.0, hi = len;
    const double A = e[0] * e[0] + e[1] * e[1];
    if (A > 0.0) {
        const double B = a[0] * e[0] + a[1] * e[1];
        const double C = a[0] * a[0] + a[1] * a[1] - g.r_max_d * g.r_max_d;
        const double disc = B * B - A * C;
        if (!(disc > 0.0)) return false;
        const double sq = sqrt(disc);
        lo = fmax(lo, (-B - sq) / A);
        hi = fmin(hi, (-B + sq) / A);
    } else if (!(a[0] * a[0] + a[1] * a[1] <= g.r_max_d * g.r_max_d)) {
        return false;
    }
    if (e[2] != 0.0) {
        const double t1 = (g.h_min_d - a[2]) / e[2], t2 = (g.h_max_d - a[2]) / e[2];
        lo = fmax(lo, fmin(t1, t2));
        hi = fmin(hi, fmax(t1, t2));
    } else if (!(a[2] >= g.h_min_d && a[2] <= g.h_max_d)) {
        return false;
    }
    if (!(hi >= lo)) return false;
    const double kmax = ceil(len / step - 0.5) - 1.0;  // last sample with d_k < len
    const double k0 = fmax(0.0, floor(lo / step - 0.5) - 1.0);
    const double k1 = fmin(kmax, ceil(hi / step - 0.5) + 1.0);
    if (!(k1 >= k0)) return false;
    kb = k0;
    n = (int)(k1 - k0) + 1;
    return true;
}

// One thread per pixel of views [view_begin, view_begin + gridDim.y).
// SART = false: proj[view] = q.  SART = true: rho[pixel] = wp (p - q) / L
// (0 where L = 0) for one view (gridDim.y = 1), p read from proj.
template <bool LINEAR, bool SART, int VT>
__global__ __launch_bounds__(256) void fp_sampled_kernel(const GeomDev g, const void *__restrict__ vol,
                                                         void *__restrict__ proj, int pt, const void *__restrict__ pw,
                                                         int pwt, float *__restrict__ rho, int view_begin,
                                                         double step) {
    const int view = view_begin + (int)blockIdx.y;
    const int pix = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (pix >= g.rows * g.cols) return;
    const int v = pix / g.cols, u = pix % g.cols;
    const ViewDev &V = g.views[view];
    double e[3];
    for (int i = 0; i < 3; ++i) e[i] = fma((double)v, V.V[i], fma((double)u, V.U[i], V.d0[i]));
    const double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int i = 0; i < 3; ++i) e[i] /= len;
    float q = 0.0f;
    int count = 0;
    double kb;
    int ns;
    if (sample_range(g, V.a, e, len, step, kb, ns)) {
        const double d0 = (kb + 0.5) * step;
        const float x0 = (float)(V.a[0] + d0 * e[0]), y0 = (float)(V.a[1] + d0 * e[1]),
                    z0 = (float)(V.a[2] + d0 * e[2]);
        const float sx = (float)(step * e[0]), sy = (float)(step * e[1]), sz = (float)(step * e[2]);
        const float two_pi = 6.28318530717958647692f;
        for (int k = 0; k < ns; ++k) {
            const float fk = (float)k;
            const float x = fmaf(fk, sx, x0), y = fmaf(fk, sy, y0), z = fmaf(fk, sz, z0);
            const float r = sqrtf(x * x + y * y);
            if (!(r >= g.r_min && r < (float)g.r_max_d && z >= g.h_min && z < (float)g.h_max_d)) continue;
            ++count;
            float th = atan2f(y, x) - g.theta0;
            th -= two_pi * floorf(th * (1.0f / two_pi));
            if (!LINEAR) {
                const int ir = clampi((int)floorf((r - g.r_min) * g.inv_dr), 0, g.n_r - 1);
                const int ih = clampi((int)floorf((z - g.h_min) * g.inv_dh), 0, g.n_h - 1);
                const int it = clampi((int)floorf(th * g.inv_dtheta), 0, g.n_theta - 1);
                q += ld_any(vol, VT, ((size_t)ih * g.n_theta + it) * g.n_r + ir);
            } else {
                const float fr = (r - g.r_min) * g.inv_dr - 0.5f;
                const float fh = (z - g.h_min) * g.inv_dh - 0.5f;
                const float ft = th * g.inv_dtheta - 0.5f;
                const float r0f = floorf(fr), h0f = floorf(fh), t0f = floorf(ft);
                const float wr = fr - r0f, wh = fh - h0f, wt = ft - t0f;
                const int r0 = (int)r0f, h0 = (int)h0f, t0 = (int)t0f;
                float acc = 0.0f;
                for (int dh = 0; dh < 2; ++dh) {
                    const int ih = clampi(h0 + dh, 0, g.n_h - 1);
                    const float whh = dh ? wh : 1.0f - wh;
                    for (int dt = 0; dt < 2; ++dt) {
                        // t0 lies in [-1, n_theta - 1]: wrap by one period either way
                        int it = t0 + dt;
                        it += it < 0 ? g.n_theta : 0;
                        it -= it >= g.n_theta ? g.n_theta : 0;
                        const float wtt = dt ? wt : 1.0f - wt;
                        const size_t rowb = ((size_t)ih * g.n_theta + it) * g.n_r;
                        const float a0 = ld_any(vol, VT, rowb + clampi(r0, 0, g.n_r - 1));
                        const float a1 = ld_any(vol, VT, rowb + clampi(r0 + 1, 0, g.n_r - 1));
                        acc = fmaf(whh * wtt, fmaf(wr, a1 - a0, a0), acc);
                    }
                }
                q += acc;
            }
        }
    }
    const float sf = (float)step;
    q *= sf;
    const size_t o = ((size_t)view * g.rows + v) * g.cols + u;
    if (!SART) {
        st_any(proj, pt, o, q);
    } else {
        const float L = sf * (float)count;
        const float w = pw ? ld_any(pw, pwt, o) : 1.0f;
        rho[pix] = L > 0.0f ? w * (ld_any(proj, pt, o) - q) / L : 0.0f;
    }
}

// One thread per cell.  MODE 0: vol = (accumulate ? vol : 0) + sum over the
// views of the bilinear reading of y at the cell centre's projection.
// MODE 1 (SART, one view, y = FP32 residual image): vol += lam wv c / n with n
// the bilinear weights that fell on the detector.
template <int MODE>
__global__ __launch_bounds__(256) void bp_voxel_kernel(const GeomDev g, const void *__restrict__ y, int yt,
                                                       void *__restrict__ vol, int vt, const void *__restrict__ vw,
                                                       int vwt, int view_begin, int view_end, int accumulate,
                                                       float lam, int nonneg) {
    const size_t ncell = (size_t)g.n_h * g.n_theta * g.n_r;
    const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ncell) return;
    const int ir = (int)(m % g.n_r), it = (int)((m / g.n_r) % g.n_theta), ih = (int)(m / ((size_t)g.n_r * g.n_theta));
    const float rc = g.r_min + ((float)ir + 0.5f) * g.dr;
    const float tc = g.theta0 + ((float)it + 0.5f) * g.dtheta;
    const float hc = g.h_min + ((float)ih + 0.5f) * g.dh;
    float sn, cs;
    sincosf(tc, &sn, &cs);
    const float px = rc * cs, py = rc * sn, pz = hc;
    float c = 0.0f, n = 0.0f;
    for (int k = view_begin; k < view_end; ++k) {
        const ViewDev &V = g.views[k];
        const float X = px - V.af[0], Y = py - V.af[1], Z = pz - V.af[2];
        const float lm = V.Qi[0] * X + V.Qi[1] * Y + V.Qi[2] * Z;
        if (!(lm > 0.0f)) continue;
        const float u = (V.Qi[3] * X + V.Qi[4] * Y + V.Qi[5] * Z) / lm;
        const float v = (V.Qi[6] * X + V.Qi[7] * Y + V.Qi[8] * Z) / lm;
        if (!(u > -1.0f && u < (float)g.cols && v > -1.0f && v < (float)g.rows)) continue;
        const float u0f = floorf(u), v0f = floorf(v);
        const float fu = u - u0f, fv = v - v0f;
        const int u0 = (int)u0f, v0 = (int)v0f;
        const size_t base = MODE == 1 ? 0 : (size_t)(k - view_begin) * g.rows * g.cols;
        for (int dv = 0; dv < 2; ++dv) {
            const int vv = v0 + dv;
            if (vv < 0 || vv >= g.rows) continue;
            const float wv_ = dv ? fv : 1.0f - fv;
            for (int du = 0; du < 2; ++du) {
                const int uu = u0 + du;
                if (uu < 0 || uu >= g.cols) continue;
                const float w = wv_ * (du ? fu : 1.0f - fu);
                c = fmaf(w, ld_any(y, yt, base + (size_t)vv * g.cols + uu), c);
                n += w;
            }
        }
    }
    if (MODE == 0) {
        st_any(vol, vt, m, (accumulate ? ld_any(vol, vt, m) : 0.0f) + c);
    } else if (n > 0.0f) {
        const float w = vw ? ld_any(vw, vwt, m) : 1.0f;
        float mu = ld_any(vol, vt, m) + lam * w * c / n;
        if (nonneg && mu < 0.0f) mu = 0.0f;
        st_any(vol, vt, m, mu);
    }
}

int launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    return CYL_OK;
}

struct Guard {
    int prev = -1;
    bool ok = true;
    explicit Guard(int dev) {
        hipGetDevice(&prev);
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~Guard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

template <int VT>
void launch_fp_sampled_t(const cyl_geom *G, const void *vol, void *proj, int pt, int vb, int nv, double step,
                         int interp, bool sart, const void *pw, int pwt, float *rho, hipStream_t st) {
    const int npix = G->rows * G->cols;
    for (int v0 = 0; v0 < nv; v0 += 65535) {
        const dim3 grid((npix + 255) / 256, std::min(65535, nv - v0));
#define CYL_FP_SAMPLED(LIN, SRT)                                                                               \
    hipLaunchKernelGGL((fp_sampled_kernel<LIN, SRT, VT>), grid, dim3(256), 0, st, G->dev, vol, proj, pt, pw, pwt, \
                       rho, vb + v0, step)
        if (interp) {
            if (sart)
                CYL_FP_SAMPLED(true, true);
            else
                CYL_FP_SAMPLED(true, false);
        } else {
            if (sart)
                CYL_FP_SAMPLED(false, true);
            else
                CYL_FP_SAMPLED(false, false);
        }
#undef CYL_FP_SAMPLED
    }
}

void launch_fp_sampled(const cyl_geom *G, const void *vol, int vt, void *proj, int pt, int vb, int nv, double step,
                       int interp, bool sart, const void *pw, int pwt, float *rho, hipStream_t st) {
    if (vt == CYL_F32)
        launch_fp_sampled_t<CYL_F32>(G, vol, proj, pt, vb, nv, step, interp, sart, pw, pwt, rho, st);
    else if (vt == CYL_F16)
        launch_fp_sampled_t<CYL_F16>(G, vol, proj, pt, vb, nv, step, interp, sart, pw, pwt, rho, st);
    else
        launch_fp_sampled_t<CYL_BF16>(G, vol, proj, pt, vb, nv, step, interp, sart, pw, pwt, rho, st);
}

int sampled_step_check(const cyl_geom *G, double step, int interp, const char *who) {
    if (!(step > 0.0) || !std::isfinite(step)) {
        set_error("%s: step must be positive and finite", who);
        return CYL_EINVAL;
    }
    // a ray's samples inside the support span at most its diameter
    const double diam = 2.0 * G->grid.r_max + (G->grid.h_max - G->grid.h_min);
    if (diam / step + 8.0 > 1073741824.0) {
        set_error("%s: step %g too small for a support of diameter %g", who, step, diam);
        return CYL_EINVAL;
    }
    if (interp != 0 && interp != 1) {
        set_error("%s: interp must be 0 (nearest) or 1 (linear)", who);
        return CYL_EINVAL;
    }
    return CYL_OK;
}

}  // namespace

}  // namespace cyl

using namespace cyl;

extern "C" int cyl_fp_sampled(const cyl_geom *G, const void *vol, cyl_dtype vt, void *proj, cyl_dtype pt,
                              int32_t view_begin, int32_t view_end, double step, int32_t interp, void *hip_stream) {
    if (!G || !vol || !proj) {
        set_error("cyl_fp_sampled: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_fp_sampled volume")) || (rc = check_dtype(pt, "cyl_fp_sampled projections")))
        return rc;
    if (view_begin < 0 || view_end > G->n_views || view_begin > view_end) {
        set_error("cyl_fp_sampled: view range [%d, %d) outside [0, %d)", view_begin, view_end, G->n_views);
        return CYL_EINVAL;
    }
    if ((rc = sampled_step_check(G, step, interp, "cyl_fp_sampled"))) return rc;
    if (view_begin == view_end) return CYL_OK;
    Guard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_fp_sampled: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_fp_sampled(G, vol, vt, proj, pt, view_begin, view_end - view_begin, step, interp, false, nullptr,
                      CYL_F32, nullptr, (hipStream_t)hip_stream);
    return launch_check("cyl_fp_sampled");
}

extern "C" int cyl_bp_voxel(const cyl_geom *G, const void *proj, cyl_dtype pt, void *vol, cyl_dtype vt,
                            int32_t view_begin, int32_t view_end, int32_t accumulate, void *hip_stream) {
    if (!G || !vol || !proj) {
        set_error("cyl_bp_voxel: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_bp_voxel volume")) || (rc = check_dtype(pt, "cyl_bp_voxel projections")))
        return rc;
    if (view_begin < 0 || view_end > G->n_views || view_begin > view_end) {
        set_error("cyl_bp_voxel: view range [%d, %d) outside [0, %d)", view_begin, view_end, G->n_views);
        return CYL_EINVAL;
    }
    Guard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_bp_voxel: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    const size_t ncell = (size_t)G->dev.n_h * G->dev.n_theta * G->dev.n_r;
    // views[view_begin .. view_end) of `proj` start at its view_begin image
    const void *y = (const char *)proj + (size_t)view_begin * G->rows * G->cols * dtype_size(pt);
    hipLaunchKernelGGL(bp_voxel_kernel<0>, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, G->dev, y, (int)pt, vol, (int)vt, nullptr, (int)CYL_F32, view_begin,
                       view_end, accumulate ? 1 : 0, 0.0f, 0);
    return launch_check("cyl_bp_voxel");
}

extern "C" int cyl_sart_run_sampled(const cyl_geom *G, const cyl_sart_params *P, double step, int32_t interp,
                                    const void *proj, cyl_dtype pt, const void *pw, cyl_dtype pwt, const void *vw,
                                    cyl_dtype vwt, void *vol, cyl_dtype vt, void *workspace, size_t ws_bytes,
                                    void *hip_stream) {
    if (!G || !P || !proj || !vol) {
        set_error("cyl_sart_run_sampled: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_sart_run_sampled volume")) ||
        (rc = check_dtype(pt, "cyl_sart_run_sampled projections")))
        return rc;
    if (pw && (rc = check_dtype(pwt, "cyl_sart_run_sampled projection weights"))) return rc;
    if (vw && (rc = check_dtype(vwt, "cyl_sart_run_sampled voxel weights"))) return rc;
    if ((rc = sampled_step_check(G, step, interp, "cyl_sart_run_sampled"))) return rc;
    if (P->n_iter < 0 || P->start_iter < 0 || P->start_view < 0 || P->start_view > G->n_views ||
        !std::isfinite(P->lambda)) {
        set_error("cyl_sart_run_sampled: invalid parameters");
        return CYL_EINVAL;
    }
    if (P->view_order)
        for (int i = 0; i < G->n_views; ++i)
            if (P->view_order[i] < 0 || P->view_order[i] >= G->n_views) {
                set_error("cyl_sart_run_sampled: view_order[%d] = %d out of range", i, P->view_order[i]);
                return CYL_EINVAL;
            }
    const size_t need = cyl_sart_workspace_bytes(G, P);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_sart_run_sampled: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    if (P->start_iter >= P->n_iter) return CYL_OK;
    Guard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sart_run_sampled: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    float *rho = (float *)workspace;
    const size_t ncell = (size_t)G->dev.n_h * G->dev.n_theta * G->dev.n_r;
    for (int it = P->start_iter; it < P->n_iter; ++it) {
        const int kv0 = (it == P->start_iter) ? P->start_view : 0;
        for (int kk = kv0; kk < G->n_views; ++kk) {
            const int k = P->view_order ? P->view_order[kk] : kk;
            launch_fp_sampled(G, vol, vt, const_cast<void *>(proj), pt, k, 1, step, interp, true, pw, pwt, rho, st);
            hipLaunchKernelGGL(bp_voxel_kernel<1>, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, st, G->dev,
                               (const void *)rho, (int)CYL_F32, vol, (int)vt, vw, (int)vwt, k, k + 1, 0,
                               (float)P->lambda, P->nonneg);
        }
        if ((rc = launch_check("cyl_sart_run_sampled"))) return rc;
    }
    return CYL_OK;
}
