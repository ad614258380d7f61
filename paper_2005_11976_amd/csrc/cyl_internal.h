// Internal types of libcyl shared by the host set-up and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cyl.h"

namespace cyl {

// Per-view geometry in the object frame (Eq. 1 applied once on the host, FP64).
// The ray of pixel (u, v) has direction d = d0 + u*U + v*V from the source a.
struct ViewDev {
    double a[3];   // source
    double d0[3];  // source -> centre of pixel (u, v) = (0, 0)
    double U[3];   // pixel step along a row
    double V[3];   // pixel step along a column
    float Qi[9];   // inverse of the 3x3 matrix [d0 | U | V]: (X - a) -> (lam, lam*u, lam*v)
    float af[3];   // source, FP32
};

// Everything a kernel needs about the geometry, passed by value.
struct GeomDev {
    int32_t n_h, n_theta, n_r;
    int32_t n_views, rows, cols;
    float r_min, dr, h_min, dh, theta0, dtheta;
    float inv_dr, inv_dh, inv_dtheta;
    float dr_lo, dh_lo;  // dr - (float)dr, dh - (float)dh
    double r_min_d, r_max_d, h_min_d, h_max_d;
    const float2 *r_tab;   // n_r + 1 shell radii as (hi, lo) float pairs
    const float2 *h_tab;   // n_h + 1 axial planes as (hi, lo)
    const float2 *cs_tab;  // n_theta + 1 sector edges as (cos, sin)
    const double2 *cs64;   // the same in FP64 (ill-conditioned crossings)
    const ViewDev *views;  // n_views
    // forward-projection dispatch order for 1, 2 and 4 pieces per ray:
    // fp_order[i][blockIdx.x] = pixel tile (row-major over tiles)
    const int32_t *fp_order[3];
    // back-projection block decomposition (cells per block along h, theta, r)
    int32_t bh, bt, br;
    int32_t nbh, nbt, nbr;
};

constexpr size_t kMaxLds = 65536;    // grid tables (staged in LDS) are limited to kMaxLds / 2 bytes

}  // namespace cyl

struct cyl_geom {
    int device;
    cyl_grid grid;
    int32_t n_views, rows, cols;
    cyl::GeomDev dev;
    void *dmem;  // single device allocation holding tables and views
};

namespace cyl {
// Records the exact pieces of every ray of one view (count pass with cells
// null, then fill pass at rowptr offsets); see record_kernel.
int launch_record(const cyl_geom *G, int view, const int32_t *rowptr, int32_t *counts, int32_t *cells, float *lens,
                  float *rowsum, hipStream_t st);
void set_error(const char *fmt, ...);
int check_dtype(cyl_dtype t, const char *what);
size_t dtype_size(cyl_dtype t);
}  // namespace cyl
