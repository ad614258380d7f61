// Precomputed system matrix for scans whose views are one view rotated about
// the object axis by whole sectors (an unposed circular scan whose view step
// is a multiple of the sector angle): the acceleration by system-matrix reuse
// that the posed method gives up (Sec. 2, the references on cylindrical
// reconstruction; Eq. 6 for the entries).  Rotating a view by s sectors maps
// the ray of pixel j to a ray that meets cell (h, t + s, r) wherever the
// original met (h, t, r), with the same lengths, so view 0's exact rows
// t_jl (from the traversal) serve every view through a theta shift.
//
// Storage (device, built once): view 0's rows (CSR: per ray, cells and
// lengths in walk order, and the closed-form row sums L_j) and columns (CSC:
// per cell, the rays meeting it sorted by ray index, with the column sums
// n_m).  The forward projection reads a row per wave with the shifted cells;
// the SART update reads, for each cell m of view k, the column of the cell
// shifted back to view 0.  Both sum in a fixed order (deterministic).

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "cyl_internal.h"
#include "cyl_store.h"

struct cyl_sym {
    const cyl_geom *geom;
    int device;
    int64_t nnz, ncell;
    int32_t nrays;
    std::vector<int32_t> shift;  // per view: theta shift in sectors relative to view 0
    int32_t *rowptr;             // nrays + 1
    int32_t *rcell;              // nnz: cell index with its theta part removed (h nt nr + r)
    uint16_t *rtheta;            // nnz: the theta index
    float *rlen;                 // nnz
    float *rowsum;               // nrays
    int32_t *colptr;             // ncell + 1
    int32_t *cray;               // nnz
    float *clen;                 // nnz
    float *colsum;               // ncell
};

namespace cyl {

namespace {

// Cell index with its theta index moved by s sectors (0 <= s < nt).
__device__ __forceinline__ int32_t shifted(int32_t cell, int s, int nt, int nr) {
    const int32_t rest = cell / nr;  // h nt + t
    const int32_t t = rest % nt;
    const int32_t t2 = t + s >= nt ? t + s - nt : t + s;
    return cell + (t2 - t) * nr;
}

// Rows, after the columns are built: split each cell index into its theta
// index and the rest, so a theta shift needs no division per entry.
__global__ __launch_bounds__(256) void row_split_kernel(int64_t nnz, int nt, int nr, int32_t *__restrict__ rcell,
                                                        uint16_t *__restrict__ rtheta) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = rcell[i];
        const int32_t t = (c / nr) % nt;
        rtheta[i] = (uint16_t)t;
        rcell[i] = c - t * nr;
    }
}

// Column pass 1: cells' entry counts.
__global__ __launch_bounds__(256) void col_count_kernel(int64_t nnz, const int32_t *__restrict__ rcell,
                                                        int32_t *__restrict__ cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[rcell[i]], 1);
}

// Column pass 2: scatter (ray, length) of every row entry to its column (one
// thread per ray; slots taken with an atomic cursor, sorted afterwards).
__global__ __launch_bounds__(256) void col_fill_kernel(int nrays, const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ rcell,
                                                       const float *__restrict__ rlen, int32_t *__restrict__ cursor,
                                                       int32_t *__restrict__ cray, float *__restrict__ clen) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= nrays) return;
    for (int32_t e = rowptr[j]; e < rowptr[j + 1]; ++e) {
        const int32_t pos = atomicAdd(&cursor[rcell[e]], 1);
        cray[pos] = j;
        clen[pos] = rlen[e];
    }
}

// Column pass 3: sort each column by ray index (insertion sort; columns are
// short) and sum it in that order.
__global__ __launch_bounds__(256) void col_sort_kernel(int64_t ncell, const int32_t *__restrict__ colptr,
                                                       int32_t *__restrict__ cray, float *__restrict__ clen,
                                                       float *__restrict__ colsum) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ncell) return;
    const int32_t b = colptr[m], e = colptr[m + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        const int32_t rj = cray[i];
        const float lj = clen[i];
        int32_t k = i - 1;
        while (k >= b && cray[k] > rj) {
            cray[k + 1] = cray[k];
            clen[k + 1] = clen[k];
            --k;
        }
        cray[k + 1] = rj;
        clen[k + 1] = lj;
    }
    float n = 0.0f;
    for (int32_t i = b; i < e; ++i) n += clen[i];
    colsum[m] = n;
}

// One wave per ray of view `view` (theta shift s): q_j = sum t mu[shifted cell].
// SART: rho[pix] = wp (p - q) / L_j (0 where L_j = 0); else proj[view][pix] = q.
template <bool SART>
__global__ __launch_bounds__(256) void sym_fp_kernel(const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ rcell,
                                                     const uint16_t *__restrict__ rtheta,
                                                     const float *__restrict__ rlen,
                                                     const float *__restrict__ rowsum, int nrays, int nt, int nr,
                                                     const void *__restrict__ vol, int vt, void *__restrict__ proj,
                                                     int pt, const void *__restrict__ pw, int pwt,
                                                     float *__restrict__ rho, int view, int s) {
    const int j = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (j >= nrays) return;
    const int32_t b = rowptr[j], e = rowptr[j + 1];
    float acc = 0.0f;
    for (int32_t i = b + lane; i < e; i += 64) {
        const int t = (int)rtheta[i] + s;
        acc = fmaf(rlen[i], ld_any(vol, vt, (size_t)rcell[i] + (size_t)(t >= nt ? t - nt : t) * nr), acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane != 0) return;
    const size_t o = (size_t)view * nrays + j;
    if (!SART) {
        st_any(proj, pt, o, acc);
    } else {
        const float L = rowsum[j];
        const float w = pw ? ld_any(pw, pwt, o) : 1.0f;
        rho[j] = L > 0.0f ? w * (ld_any(proj, pt, o) - acc) / L : 0.0f;
    }
}

// One thread per cell m of view k (theta shift s): its column is that of the
// cell shifted back by s in view 0; mu_m += lam wv c / n where n > 0.
__global__ __launch_bounds__(256) void sym_update_kernel(const int32_t *__restrict__ colptr,
                                                         const int32_t *__restrict__ cray,
                                                         const float *__restrict__ clen,
                                                         const float *__restrict__ colsum, int64_t ncell, int nt,
                                                         int nr, const float *__restrict__ rho, void *__restrict__ vol,
                                                         int vt, const void *__restrict__ vw, int vwt, float lam,
                                                         int nonneg, int s_back) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ncell) return;
    const int32_t m0 = shifted((int32_t)m, s_back, nt, nr);
    const float n = colsum[m0];
    if (!(n > 0.0f)) return;
    const float w = vw ? ld_any(vw, vwt, m) : 1.0f;
    const float mu0 = ld_any(vol, vt, m);
    // the column's entries in order, eight loaded at a time (rays and lengths,
    // then the residual gathers) so their latencies overlap
    const int32_t b = colptr[m0], e = colptr[m0 + 1];
    float c = 0.0f;
    for (int32_t i0 = b; i0 < e; i0 += 8) {
        int32_t ray[8];
        float len[8], y[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ray[q] = i0 + q < e ? cray[i0 + q] : 0;
            len[q] = i0 + q < e ? clen[i0 + q] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) y[q] = i0 + q < e ? rho[ray[q]] : 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (i0 + q < e) c = fmaf(len[q], y[q], c);
    }
    float mu = mu0 + lam * w * c / n;
    if (nonneg && mu < 0.0f) mu = 0.0f;
    st_any(vol, vt, m, mu);
}

int sym_check_launch(const char *what) {
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

void free_sym(cyl_sym *S) {
    if (!S) return;
    void *p[] = {S->rowptr, S->rcell, S->rtheta, S->rlen, S->rowsum, S->colptr, S->cray, S->clen, S->colsum};
    for (void *q : p)
        if (q) hipFree(q);
    delete S;
}

// Rotation of view 0 onto view k by whole sectors: shift[k] = s if
// Rz(s dtheta) maps view 0's source, detector origin and pixel steps onto view
// k's within 1e-9 of their size (object frame).
bool view_shifts(const cyl_geom *G, const std::vector<ViewDev> &v, std::vector<int32_t> &shift, int &bad) {
    const int nt = G->dev.n_theta;
    const double dth = 2.0 * M_PI / nt;
    shift.assign(v.size(), 0);
    auto rot = [](double c, double s, const double *x, double *y) {
        y[0] = c * x[0] - s * x[1];
        y[1] = s * x[0] + c * x[1];
        y[2] = x[2];
    };
    const double *a0 = v[0].a;
    const double ang0 = std::atan2(a0[1], a0[0]);
    for (size_t k = 0; k < v.size(); ++k) {
        const double *ak = v[k].a;
        double phi = std::atan2(ak[1], ak[0]) - ang0;
        long s = std::lround(phi / dth);
        s = ((s % nt) + nt) % nt;
        const double c = std::cos(s * dth), sn = std::sin(s * dth);
        const double *src[4] = {v[0].a, v[0].d0, v[0].U, v[0].V};
        const double *dst[4] = {v[k].a, v[k].d0, v[k].U, v[k].V};
        for (int q = 0; q < 4; ++q) {
            double y[3];
            rot(c, sn, src[q], y);
            const double scale = std::sqrt(src[q][0] * src[q][0] + src[q][1] * src[q][1] + src[q][2] * src[q][2]);
            for (int i = 0; i < 3; ++i)
                if (std::fabs(y[i] - dst[q][i]) > 1e-9 * std::max(scale, 1.0)) {
                    bad = (int)k;
                    return false;
                }
        }
        shift[k] = (int32_t)s;
    }
    return true;
}

}  // namespace

}  // namespace cyl

using namespace cyl;

extern "C" int cyl_sym_create(const cyl_geom *G, cyl_sym **out, void *hip_stream) {
    if (!G || !out) {
        set_error("cyl_sym_create: NULL argument");
        return CYL_EINVAL;
    }
    *out = nullptr;
    Guard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sym_create: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<ViewDev> views(G->n_views);
    if (hipMemcpy(views.data(), G->dev.views, sizeof(ViewDev) * views.size(), hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("cyl_sym_create: cannot read the views");
        return CYL_EDEVICE;
    }
    std::vector<int32_t> shift;
    int bad = -1;
    if (!view_shifts(G, views, shift, bad)) {
        set_error("cyl_sym_create: view %d is not view 0 rotated about the object axis by whole sectors", bad);
        return CYL_EINVAL;
    }
    if (G->dev.n_theta > 65535) {
        set_error("cyl_sym_create: n_theta = %d above 65535", G->dev.n_theta);
        return CYL_EUNSUPPORTED;
    }
    cyl_sym *S = new (std::nothrow) cyl_sym();
    if (!S) {
        set_error("cyl_sym_create: out of host memory");
        return CYL_ENOMEM;
    }
    S->geom = G;
    S->device = G->device;
    S->shift = shift;
    S->nrays = G->rows * G->cols;
    S->ncell = (int64_t)G->dev.n_h * G->dev.n_theta * G->dev.n_r;
    const int32_t nrays = S->nrays;
    auto fail = [&](const char *what) {
        set_error("cyl_sym_create: %s", what);
        free_sym(S);
        return CYL_ENOMEM;
    };
    if (hipMalloc(&S->rowptr, sizeof(int32_t) * (nrays + 1)) != hipSuccess ||
        hipMalloc(&S->rowsum, sizeof(float) * nrays) != hipSuccess)
        return fail("device allocation failed (rows)");
    int32_t *counts = nullptr;
    if (hipMalloc(&counts, sizeof(int32_t) * nrays) != hipSuccess) return fail("device allocation failed (counts)");
    int rc = launch_record(G, 0, nullptr, counts, nullptr, nullptr, S->rowsum, st);
    std::vector<int32_t> hc(nrays);
    if (rc || hipMemcpyAsync(hc.data(), counts, sizeof(int32_t) * nrays, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        hipFree(counts);
        free_sym(S);
        set_error("cyl_sym_create: counting the rows failed");
        return CYL_EDEVICE;
    }
    hipFree(counts);
    std::vector<int32_t> rp(nrays + 1, 0);
    int64_t nnz = 0;
    for (int32_t j = 0; j < nrays; ++j) {
        rp[j] = (int32_t)std::min<int64_t>(nnz, INT32_MAX);
        nnz += hc[j];
    }
    if (nnz >= INT32_MAX) {
        free_sym(S);
        set_error("cyl_sym_create: %lld matrix entries per view exceed 2^31 - 1", (long long)nnz);
        return CYL_EUNSUPPORTED;
    }
    rp[nrays] = (int32_t)nnz;
    S->nnz = nnz;
    const size_t ne = (size_t)std::max<int64_t>(nnz, 1);
    if (hipMalloc(&S->rcell, sizeof(int32_t) * ne) != hipSuccess || hipMalloc(&S->rlen, sizeof(float) * ne) != hipSuccess ||
        hipMalloc(&S->rtheta, sizeof(uint16_t) * ne) != hipSuccess ||
        hipMalloc(&S->cray, sizeof(int32_t) * ne) != hipSuccess || hipMalloc(&S->clen, sizeof(float) * ne) != hipSuccess ||
        hipMalloc(&S->colptr, sizeof(int32_t) * (S->ncell + 1)) != hipSuccess ||
        hipMalloc(&S->colsum, sizeof(float) * S->ncell) != hipSuccess)
        return fail("device allocation failed (matrix)");
    if (hipMemcpyAsync(S->rowptr, rp.data(), sizeof(int32_t) * (nrays + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
        (rc = launch_record(G, 0, S->rowptr, nullptr, S->rcell, S->rlen, nullptr, st))) {
        free_sym(S);
        set_error("cyl_sym_create: filling the rows failed");
        return CYL_EDEVICE;
    }
    // columns: counts, host prefix sum, scatter, per-column sort
    int32_t *cnt = nullptr;
    if (hipMalloc(&cnt, sizeof(int32_t) * S->ncell) != hipSuccess) return fail("device allocation failed (columns)");
    hipMemsetAsync(cnt, 0, sizeof(int32_t) * S->ncell, st);
    const unsigned egrid = (unsigned)std::min<int64_t>((nnz + 255) / 256 + 1, 1 << 20);
    hipLaunchKernelGGL(col_count_kernel, dim3(egrid), dim3(256), 0, st, nnz, S->rcell, cnt);
    std::vector<int32_t> hcnt(S->ncell);
    if ((rc = sym_check_launch("cyl_sym_create")) ||
        hipMemcpyAsync(hcnt.data(), cnt, sizeof(int32_t) * S->ncell, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        hipFree(cnt);
        free_sym(S);
        set_error("cyl_sym_create: counting the columns failed");
        return CYL_EDEVICE;
    }
    std::vector<int32_t> cp(S->ncell + 1);
    int64_t acc = 0;
    for (int64_t m = 0; m < S->ncell; ++m) {
        cp[m] = (int32_t)acc;
        acc += hcnt[m];
    }
    cp[S->ncell] = (int32_t)acc;
    hipMemcpyAsync(S->colptr, cp.data(), sizeof(int32_t) * (S->ncell + 1), hipMemcpyHostToDevice, st);
    hipMemcpyAsync(cnt, cp.data(), sizeof(int32_t) * S->ncell, hipMemcpyHostToDevice, st);  // cursors
    hipLaunchKernelGGL(col_fill_kernel, dim3((unsigned)((nrays + 255) / 256)), dim3(256), 0, st, nrays, S->rowptr,
                       S->rcell, S->rlen, cnt, S->cray, S->clen);
    hipLaunchKernelGGL(col_sort_kernel, dim3((unsigned)((S->ncell + 255) / 256)), dim3(256), 0, st, S->ncell,
                       S->colptr, S->cray, S->clen, S->colsum);
    hipLaunchKernelGGL(row_split_kernel, dim3(egrid), dim3(256), 0, st, nnz, G->dev.n_theta, G->dev.n_r, S->rcell,
                       S->rtheta);
    rc = sym_check_launch("cyl_sym_create");
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = CYL_EDEVICE;
    hipFree(cnt);
    if (rc) {
        free_sym(S);
        return rc;
    }
    *out = S;
    return CYL_OK;
}

extern "C" void cyl_sym_destroy(cyl_sym *S) {
    if (!S) return;
    Guard dg(S->device);
    free_sym(S);
}

extern "C" int64_t cyl_sym_nnz(const cyl_sym *S) { return S ? S->nnz : -1; }

extern "C" int cyl_sym_fp(const cyl_sym *S, const void *vol, cyl_dtype vt, void *proj, cyl_dtype pt,
                          int32_t view_begin, int32_t view_end, void *hip_stream) {
    if (!S || !vol || !proj) {
        set_error("cyl_sym_fp: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_sym_fp volume")) || (rc = check_dtype(pt, "cyl_sym_fp projections"))) return rc;
    const cyl_geom *G = S->geom;
    if (view_begin < 0 || view_end > G->n_views || view_begin > view_end) {
        set_error("cyl_sym_fp: view range [%d, %d) outside [0, %d)", view_begin, view_end, G->n_views);
        return CYL_EINVAL;
    }
    Guard dg(S->device);
    const dim3 grid((unsigned)((S->nrays + 3) / 4));
    for (int k = view_begin; k < view_end; ++k)
        hipLaunchKernelGGL(sym_fp_kernel<false>, grid, dim3(256), 0, (hipStream_t)hip_stream, S->rowptr, S->rcell,
                           S->rtheta, S->rlen, S->rowsum, S->nrays, G->dev.n_theta, G->dev.n_r, vol, (int)vt, proj, (int)pt,
                           nullptr, (int)CYL_F32, nullptr, k, S->shift[k]);
    return sym_check_launch("cyl_sym_fp");
}

extern "C" int cyl_sym_sart_run(const cyl_sym *S, const cyl_sart_params *P, const void *proj, cyl_dtype pt,
                                const void *pw, cyl_dtype pwt, const void *vw, cyl_dtype vwt, void *vol, cyl_dtype vt,
                                void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!S || !P || !proj || !vol) {
        set_error("cyl_sym_sart_run: NULL argument");
        return CYL_EINVAL;
    }
    const cyl_geom *G = S->geom;
    int rc;
    if ((rc = check_dtype(vt, "cyl_sym_sart_run volume")) || (rc = check_dtype(pt, "cyl_sym_sart_run projections")))
        return rc;
    if (pw && (rc = check_dtype(pwt, "cyl_sym_sart_run projection weights"))) return rc;
    if (vw && (rc = check_dtype(vwt, "cyl_sym_sart_run voxel weights"))) return rc;
    if (P->n_iter < 0 || P->start_iter < 0 || P->start_view < 0 || P->start_view > G->n_views ||
        !std::isfinite(P->lambda)) {
        set_error("cyl_sym_sart_run: invalid parameters");
        return CYL_EINVAL;
    }
    if (P->view_order)
        for (int i = 0; i < G->n_views; ++i)
            if (P->view_order[i] < 0 || P->view_order[i] >= G->n_views) {
                set_error("cyl_sym_sart_run: view_order[%d] = %d out of range", i, P->view_order[i]);
                return CYL_EINVAL;
            }
    const size_t need = cyl_sart_workspace_bytes(G, P);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_sym_sart_run: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    if (P->start_iter >= P->n_iter) return CYL_OK;
    Guard dg(S->device);
    hipStream_t st = (hipStream_t)hip_stream;
    float *rho = (float *)workspace;
    const int nt = G->dev.n_theta, nr = G->dev.n_r;
    const dim3 fgrid((unsigned)((S->nrays + 3) / 4)), ugrid((unsigned)((S->ncell + 255) / 256));
    for (int it = P->start_iter; it < P->n_iter; ++it) {
        const int kv0 = (it == P->start_iter) ? P->start_view : 0;
        for (int kk = kv0; kk < G->n_views; ++kk) {
            const int k = P->view_order ? P->view_order[kk] : kk;
            const int s = S->shift[k];
            hipLaunchKernelGGL(sym_fp_kernel<true>, fgrid, dim3(256), 0, st, S->rowptr, S->rcell, S->rtheta, S->rlen,
                               S->rowsum,
                               S->nrays, nt, nr, vol, (int)vt, const_cast<void *>(proj), (int)pt, pw, (int)pwt, rho,
                               k, s);
            hipLaunchKernelGGL(sym_update_kernel, ugrid, dim3(256), 0, st, S->colptr, S->cray, S->clen, S->colsum,
                               S->ncell, nt, nr, (const float *)rho, vol, (int)vt, vw, (int)vwt, (float)P->lambda,
                               P->nonneg, s == 0 ? 0 : nt - s);
        }
        if ((rc = sym_check_launch("cyl_sym_sart_run"))) return rc;
    }
    return CYL_OK;
}
