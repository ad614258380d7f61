// Host side of libcyl: argument validation, FP64 geometry precompute (Eq. 1
// applied once per view), grid tables, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "cyl_internal.h"

namespace cyl {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_dtype(cyl_dtype t, const char *what) {
    if (t != CYL_F32 && t != CYL_F16 && t != CYL_BF16) {
        set_error("%s: unsupported dtype %d", what, (int)t);
        return CYL_EINVAL;
    }
    return CYL_OK;
}

size_t dtype_size(cyl_dtype t) { return t == CYL_F32 ? 4 : 2; }

static bool finite3(const double *v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

static void mat_vec(const double R[9], const double x[3], double out[3]) {
    for (int i = 0; i < 3; ++i) out[i] = R[3 * i] * x[0] + R[3 * i + 1] * x[1] + R[3 * i + 2] * x[2];
}

// Inverse of the 3x3 matrix with columns c0, c1, c2; false if singular.
static bool inverse_cols(const double c0[3], const double c1[3], const double c2[3], double inv[9]) {
    double m[9] = {c0[0], c1[0], c2[0], c0[1], c1[1], c2[1], c0[2], c1[2], c2[2]};
    double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                 m[2] * (m[3] * m[7] - m[4] * m[6]);
    double scale = 1.0;
    for (int i = 0; i < 3; ++i) scale *= std::sqrt(c0[i] * c0[i] + c1[i] * c1[i] + c2[i] * c2[i]) + 1e-300;
    if (!(std::fabs(det) > 1e-12 * scale)) return false;
    double id = 1.0 / det;
    inv[0] = (m[4] * m[8] - m[5] * m[7]) * id;
    inv[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    inv[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    inv[3] = (m[5] * m[6] - m[3] * m[8]) * id;
    inv[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    inv[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    inv[6] = (m[3] * m[7] - m[4] * m[6]) * id;
    inv[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    inv[8] = (m[0] * m[4] - m[1] * m[3]) * id;
    return true;
}

static float2 split(double x) {
    float hi = (float)x;
    float lo = (float)(x - (double)hi);
    return make_float2(hi, lo);
}

}  // namespace cyl

using namespace cyl;

extern "C" const char *cyl_last_error(void) { return g_err; }

extern "C" const char *cyl_version(void) { return "libcyl 0.1 (gfx950)"; }

extern "C" int cyl_geom_create(const cyl_grid *grid, const cyl_traj *traj, const cyl_pose *pose,
                               int device, cyl_geom **out) {
    if (!grid || !traj || !pose || !out) {
        set_error("cyl_geom_create: NULL argument");
        return CYL_EINVAL;
    }
    const cyl_grid g = *grid;
    if (g.n_h < 1 || g.n_theta < 1 || g.n_r < 1) {
        set_error("cyl_geom_create: grid sizes must be >= 1 (got %d x %d x %d)", g.n_h, g.n_theta, g.n_r);
        return CYL_EINVAL;
    }
    if ((int64_t)g.n_h * g.n_theta * g.n_r >= ((int64_t)1 << 30) || (int64_t)g.n_theta * g.n_r >= (1 << 24)) {
        set_error("cyl_geom_create: grid of %d x %d x %d cells exceeds 2^30 - 1 cells or n_theta * n_r >= 2^24",
                  g.n_h, g.n_theta, g.n_r);
        return CYL_EINVAL;
    }
    if (!(std::isfinite(g.r_min) && std::isfinite(g.r_max) && std::isfinite(g.h_min) &&
          std::isfinite(g.h_max) && std::isfinite(g.theta0))) {
        set_error("cyl_geom_create: non-finite grid extent");
        return CYL_EINVAL;
    }
    if (!(g.r_min >= 0.0 && g.r_min < g.r_max)) {
        set_error("cyl_geom_create: need 0 <= r_min < r_max (got %g, %g)", g.r_min, g.r_max);
        return CYL_EINVAL;
    }
    if (!(g.h_min < g.h_max)) {
        set_error("cyl_geom_create: need h_min < h_max (got %g, %g)", g.h_min, g.h_max);
        return CYL_EINVAL;
    }
    if (traj->n_views < 1 || traj->det_rows < 1 || traj->det_cols < 1 || !traj->views) {
        set_error("cyl_geom_create: trajectory needs n_views, det_rows, det_cols >= 1 and views");
        return CYL_EINVAL;
    }
    if ((int64_t)traj->det_rows * traj->det_cols > (int64_t)1 << 28 || traj->det_rows > 32767 ||
        traj->det_cols > 65535) {
        set_error("cyl_geom_create: detector larger than 2^28 pixels, 32767 rows or 65535 columns");
        return CYL_EINVAL;
    }
    // pose must be a rotation
    const double *R = pose->R;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(R[i])) {
            set_error("cyl_geom_create: non-finite rotation");
            return CYL_EINVAL;
        }
    if (!finite3(pose->T)) {
        set_error("cyl_geom_create: non-finite translation");
        return CYL_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dot = R[3 * i] * R[3 * j] + R[3 * i + 1] * R[3 * j + 1] + R[3 * i + 2] * R[3 * j + 2];
            if (std::fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-9) {
                set_error("cyl_geom_create: R is not orthonormal");
                return CYL_EINVAL;
            }
        }
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                 R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det < 0.0) {
        set_error("cyl_geom_create: R is a reflection (det < 0)");
        return CYL_EINVAL;
    }
    const size_t table_bytes = 8 * ((size_t)(g.n_r + 1) + (g.n_h + 1) + (g.n_theta + 1));
    if (table_bytes > kMaxLds / 2) {
        set_error("cyl_geom_create: grid tables of %zu bytes exceed the %zu-byte LDS budget "
                  "(n_r + n_h + n_theta must stay below %zu)", table_bytes, kMaxLds / 2, kMaxLds / 16 - 3);
        return CYL_EUNSUPPORTED;
    }
    int ndev = 0;
    // per-view object-frame geometry (Eq. 1, FP64)
    const int nv = traj->n_views, H = traj->det_rows, W = traj->det_cols;
    std::vector<ViewDev> views(nv);
    const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
    for (int k = 0; k < nv; ++k) {
        const double *w = traj->views + 12 * (size_t)k;
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(w[i])) {
                set_error("cyl_geom_create: view %d has a non-finite entry", k);
                return CYL_EINVAL;
            }
        double S[3], D[3], U[3], V[3];
        mat_vec(R, w, S);
        mat_vec(R, w + 3, D);
        mat_vec(R, w + 6, U);
        mat_vec(R, w + 9, V);
        for (int i = 0; i < 3; ++i) {
            S[i] += pose->T[i];
            D[i] += pose->T[i];
        }
        ViewDev &vd = views[k];
        for (int i = 0; i < 3; ++i) {
            vd.a[i] = S[i];
            vd.U[i] = U[i];
            vd.V[i] = V[i];
            vd.d0[i] = D[i] - cu * U[i] - cv * V[i] - S[i];
            vd.af[i] = (float)S[i];
        }
        // source must be outside the grid support
        double rs = std::hypot(S[0], S[1]);
        if (rs < g.r_max && S[2] >= g.h_min && S[2] < g.h_max) {
            set_error("cyl_geom_create: source of view %d lies inside the grid support", k);
            return CYL_EINVAL;
        }
        double Qi[9];
        if (!inverse_cols(vd.d0, vd.U, vd.V, Qi)) {
            set_error("cyl_geom_create: view %d has a degenerate detector", k);
            return CYL_EINVAL;
        }
        for (int i = 0; i < 9; ++i) vd.Qi[i] = (float)Qi[i];
    }
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        set_error("cyl_geom_create: no HIP device (%s)", hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        set_error("cyl_geom_create: device %d out of range [0, %d)", device, ndev);
        return CYL_EINVAL;
    }
    int prev = 0;
    hipGetDevice(&prev);
    if ((e = hipSetDevice(device)) != hipSuccess) {
        set_error("cyl_geom_create: hipSetDevice(%d): %s", device, hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    // grid tables
    std::vector<float2> rt(g.n_r + 1), ht(g.n_h + 1), cs(g.n_theta + 1);
    std::vector<double2> cs64(g.n_theta + 1);
    const double dr = (g.r_max - g.r_min) / g.n_r, dh = (g.h_max - g.h_min) / g.n_h;
    const double dth = 2.0 * M_PI / g.n_theta;
    for (int i = 0; i <= g.n_r; ++i) rt[i] = split(g.r_min + i * dr);
    for (int m = 0; m <= g.n_h; ++m) ht[m] = split(g.h_min + m * dh);
    for (int b = 0; b <= g.n_theta; ++b) {
        double th = g.theta0 + b * dth;
        cs64[b] = make_double2(std::cos(th), std::sin(th));
        cs[b] = make_float2((float)cs64[b].x, (float)cs64[b].y);
    }
    // edge n_theta is edge 0 (theta0 + 2 pi), and for even n_theta edge
    // b + n_theta/2 lies on the same line as edge b: give each line a single
    // representation so that neighbouring sectors share their edges exactly
    if (g.n_theta % 2 == 0)
        for (int b = 0; b < g.n_theta / 2; ++b) {
            cs64[b + g.n_theta / 2] = make_double2(-cs64[b].x, -cs64[b].y);
            cs[b + g.n_theta / 2] = make_float2(-cs[b].x, -cs[b].y);
        }
    cs64[g.n_theta] = cs64[0];
    cs[g.n_theta] = cs[0];
    // forward-projection dispatch orders (pieces per ray 1, 2, 4: tiles 32, 16,
    // 8 pixels wide by 8 high).  Workgroups go round-robin to the 8 XCDs; XCD x
    // receives a contiguous run of row-major tiles (a band of rows, so its L2
    // holds one band of the volume) in centre-out column order: the central
    // columns carry the longest rays, so dispatching them first leaves the
    // short edge tiles for the tail of the launch.
    std::vector<int32_t> fpo[3];
    for (int i = 0; i < 3; ++i) {
        const int tw = 8 * (4 >> i);  // pieces per ray 1 << i
        const int tu = (W + tw - 1) / tw, tv = (H + 7) / 8;
        const int total = tu * tv;
        fpo[i].assign(total, 0);
        int start = 0;
        for (int x = 0; x < 8; ++x) {
            const int n = total / 8 + (x < total % 8 ? 1 : 0);
            std::vector<int32_t> list(n);
            for (int k = 0; k < n; ++k) list[k] = start + k;
            std::stable_sort(list.begin(), list.end(), [tu](int32_t a, int32_t b) {
                const double da = std::fabs(a % tu + 0.5 - 0.5 * tu), db = std::fabs(b % tu + 0.5 - 0.5 * tu);
                return da < db;
            });
            for (int k = 0; k < n; ++k) fpo[i][x + 8 * k] = list[k];
            start += n;
        }
    }
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off_views = 0;
    size_t off_r = align(off_views + sizeof(ViewDev) * nv);
    size_t off_h = align(off_r + sizeof(float2) * rt.size());
    size_t off_cs = align(off_h + sizeof(float2) * ht.size());
    size_t off_cs64 = align(off_cs + sizeof(float2) * cs.size());
    size_t off_fpo[3];
    size_t total = align(off_cs64 + sizeof(double2) * cs64.size());
    for (int i = 0; i < 3; ++i) {
        off_fpo[i] = total;
        total = align(total + sizeof(int32_t) * fpo[i].size());
    }
    void *dmem = nullptr;
    if ((e = hipMalloc(&dmem, total)) != hipSuccess) {
        hipSetDevice(prev);
        set_error("cyl_geom_create: hipMalloc(%zu): %s", total, hipGetErrorString(e));
        return CYL_ENOMEM;
    }
    char *base = (char *)dmem;
    bool ok = hipMemcpy(base + off_views, views.data(), sizeof(ViewDev) * nv, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + off_r, rt.data(), sizeof(float2) * rt.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + off_h, ht.data(), sizeof(float2) * ht.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + off_cs, cs.data(), sizeof(float2) * cs.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(base + off_cs64, cs64.data(), sizeof(double2) * cs64.size(), hipMemcpyHostToDevice) == hipSuccess;
    for (int i = 0; i < 3 && ok; ++i)
        ok = hipMemcpy(base + off_fpo[i], fpo[i].data(), sizeof(int32_t) * fpo[i].size(), hipMemcpyHostToDevice) ==
             hipSuccess;
    if (!ok) {
        hipFree(dmem);
        hipSetDevice(prev);
        set_error("cyl_geom_create: upload of the geometry tables failed");
        return CYL_EDEVICE;
    }
    cyl_geom *G = new (std::nothrow) cyl_geom;
    if (!G) {
        hipFree(dmem);
        hipSetDevice(prev);
        set_error("cyl_geom_create: out of host memory");
        return CYL_ENOMEM;
    }
    G->device = device;
    G->grid = g;
    G->n_views = nv;
    G->rows = H;
    G->cols = W;
    G->dmem = dmem;
    GeomDev &d = G->dev;
    d.n_h = g.n_h;
    d.n_theta = g.n_theta;
    d.n_r = g.n_r;
    d.n_views = nv;
    d.rows = H;
    d.cols = W;
    d.r_min = (float)g.r_min;
    d.dr = (float)dr;
    d.h_min = (float)g.h_min;
    d.dh = (float)dh;
    d.theta0 = (float)g.theta0;
    d.dtheta = (float)dth;
    d.inv_dr = (float)(1.0 / dr);
    d.inv_dh = (float)(1.0 / dh);
    d.inv_dtheta = (float)(1.0 / dth);
    d.dr_lo = (float)(dr - (double)d.dr);
    d.dh_lo = (float)(dh - (double)d.dh);
    d.r_min_d = g.r_min;
    d.r_max_d = g.r_max;
    d.h_min_d = g.h_min;
    d.h_max_d = g.h_max;
    d.views = (const ViewDev *)(base + off_views);
    d.r_tab = (const float2 *)(base + off_r);
    d.h_tab = (const float2 *)(base + off_h);
    d.cs_tab = (const float2 *)(base + off_cs);
    d.cs64 = (const double2 *)(base + off_cs64);
    for (int i = 0; i < 3; ++i) d.fp_order[i] = (const int32_t *)(base + off_fpo[i]);
    // back-projection blocks: flat in h, wide in theta and r; wedges no wider than pi
    d.bh = g.n_h < 4 ? g.n_h : 4;
    d.br = g.n_r < 16 ? g.n_r : 16;
    int bt = g.n_theta / 2;
    if (bt < 1) bt = 1;
    if (bt > 16) bt = 16;
    d.bt = bt;
    // A back-projection super-block of at most 8 such blocks needs at most
    // 32 (18 x 17 + 1) + 5 64-bit accumulator words (79 KiB, 8 blocks stacked
    // in h) beside the at most 35 sector edges it stages: well inside the
    // 160 KiB a workgroup may hold, so the block shape does not depend on N_theta.
    d.nbh = (g.n_h + d.bh - 1) / d.bh;
    d.nbt = (g.n_theta + d.bt - 1) / d.bt;
    d.nbr = (g.n_r + d.br - 1) / d.br;
    hipSetDevice(prev);
    *out = G;
    return CYL_OK;
}

extern "C" void cyl_geom_destroy(cyl_geom *geom) {
    if (!geom) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(geom->device);
    hipFree(geom->dmem);
    hipSetDevice(prev);
    delete geom;
}
