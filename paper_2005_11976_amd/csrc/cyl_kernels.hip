// HIP kernels of libcyl (gfx950): cylindrical Siddon traversal, forward
// projection with the SART residual epilogue, back-projection on shared
// super-blocks of cells (the plain transpose, or the SART update epilogue),
// closed-form row sums, and the C entry points that launch them.
//
// Ray model (Sec. 2.2, Eq. 6): one ray per pixel from the source to the pixel
// centre; t_jl is the exact length of that segment inside ring-sector cell l
// (Sec. 2, Eq. 2).  The traversal parametrises each ray by its arc length s
// (mm) measured from the point of closest approach to the object axis, so all
// FP32 crossing parameters stay small and well conditioned:
//   r-shells      r(s)^2 = b^2 + (kappa s)^2         ->  s = +-sqrt((r-b)(r+b)) / kappa
//   sector edges  n_b . (c + s e_xy) = 0             ->  s = -(n_b . c) / (n_b . e_xy)
//   axial planes  z(s) = z_c + s e_z                 ->  s = (h_m - z_c) / e_z
// b, c and z_c come from an FP64 set-up per ray; b and the table radii carry a
// second FP32 word so r - b keeps its precision at grazing incidence.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "cyl_internal.h"
#include "cyl_isa.h"
#include "cyl_block.h"
#include "cyl_ray.h"
#include "cyl_store.h"

namespace cyl {

// ------------------------------------------------------------ grid tables

__device__ __forceinline__ size_t table_floats2(const GeomDev &g) {
    return (size_t)(g.n_r + 1) + (g.n_h + 1) + (g.n_theta + 1);
}

// Cooperative copy of the grid tables (radii, planes, sector edges in the
// object frame) into LDS; the caller synchronises.
__device__ __forceinline__ Tabs stage_tables(const GeomDev &g, float2 *smem) {
    const int nr = g.n_r + 1, nh = g.n_h + 1, nc = g.n_theta + 1;
    for (int i = threadIdx.x; i < nr; i += blockDim.x) smem[i] = g.r_tab[i];
    for (int i = threadIdx.x; i < nh; i += blockDim.x) smem[nr + i] = g.h_tab[i];
    for (int i = threadIdx.x; i < nc; i += blockDim.x) smem[nr + nh + i] = g.cs_tab[i];
    Tabs T;
    T.r = smem;
    T.h = smem + nr;
    T.cs = smem + nr + nh;
    T.cs_lo = 0;
    T.cs_n = g.n_theta;
    return T;
}

// Frame of a whole-ray walk: the object frame, with the reference point
// nearest the grid centre.
__device__ __forceinline__ Frame grid_frame(const GeomDev &g) {
    Frame F;
    F.cw = 1.0;
    F.sw = 0.0;
    F.gx = F.gy = 0.0f;
    F.gz = (float)(0.5 * (g.h_min_d + g.h_max_d));
    F.wsec = -g.theta0 * g.inv_dtheta;
    return F;
}

// Minimum and maximum over the 64 lanes of a wave (all lanes active).
__device__ __forceinline__ float wave_min(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ float wave_max(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}

// Aligned 8x8 pixel tiles of a view.  The SART workspace holds, after the FP32
// residual images of an update, one float per tile and view: the largest
// |rho| of the tile, written by the residual FP and read by the update to
// bound its fixed-point sums.
__host__ __device__ __forceinline__ size_t tile_count(const GeomDev &g) {
    return (size_t)((g.rows + 7) >> 3) * (size_t)((g.cols + 7) >> 3);
}

// ------------------------------------------------------------ launch items

// One launch covers up to kMaxBatch items, each a scan (its geometry, buffers
// and views); blockIdx.y selects the item.  A single call is a launch of one
// item, a batched SART step one item per scan, so every path runs the same
// kernels.  The items travel in the kernel arguments (read with scalar loads,
// uniform across the workgroup), which bounds a launch to 16 items.
constexpr int kMaxBatch = 16;

struct FpItem {
    GeomDev g;
    const void *vol;      // volume (storage type VT)
    void *proj;           // projections: output (plain) or measured data (SART)
    const void *pw;       // SART: projection weights or null; plain: minuend or null
    float *rho;           // residual image of the view (SART)
    float *tmax;          // SART: largest |rho| of each aligned 8x8 pixel tile of the view
    int view, ns, nwg, pwt;  // view, pieces per ray, workgroups, type of pw
};
struct FpLaunch {
    int n;
    FpItem item[kMaxBatch];
};

struct BpItem {
    GeomDev g;
    const void *y;        // projections (plain) or FP32 residual images (SART), one per position
    void *vol;
    const void *vw;       // voxel weights or null (SART)
    const int32_t *views; // SART: device list of views, position k -> views[k]; null: view k
    int view_begin, view_end, nwg;
    int flags;            // bit 0: accumulate (plain), bit 1: nonneg (SART), bits 8+: type of vw
    float lam;
};
struct BpLaunch {
    int n;
    BpItem item[kMaxBatch];
};
static_assert(sizeof(FpLaunch) <= 4096 && sizeof(BpLaunch) <= 4096, "kernel arguments are limited to 4 KiB");

// ------------------------------------------------------------ forward projection

// Partial forward projection of piece `piece` of `npieces` equal parameter
// ranges of ray (u, v): each piece starts from its own cell so the pieces of
// one ray can run on neighbouring lanes.
template <int VT, bool PRECISE, bool REFINE>
__device__ __forceinline__ float fp_piece(const GeomDev &g, const Tabs &T, const ViewDev &V, const Frame &F,
                                          const Ray &r, __amdgpu_buffer_rsrc_t vol, int piece, int npieces) {
    if (!(r.flags & RAY_HIT)) return 0.0f;
    const float span = (r.s_out - r.s_in) / (float)npieces;
    const float a0 = piece == 0 ? r.s_in : fmaf((float)piece, span, r.s_in);
    const float a1 = piece == npieces - 1 ? r.s_out : fmaf((float)(piece + 1), span, r.s_in);
    if (!(a1 > a0)) return 0.0f;
    int ih, it, ir;
    cell_at(g, r, F, a0, ih, it, ir);
    // the gather of one step is consumed at the start of the next (before the
    // next gather is issued, so the two share a register and the wait for the
    // load falls a whole step later); cell indices fit in 24-bit products
    // (checked when the geometry is created)
    struct Gather {
        __amdgpu_buffer_rsrc_t vol;
        int nh, nt, nr, ntr;
        float acc, plen, pval;
        __device__ __forceinline__ void operator()(int h, int t, int q, float len) {
            // a slab index outside the grid (a step of rounding past its end
            // faces) addresses past the volume, where the buffer load reads 0;
            // the hole (q = -1) reads a neighbouring word (or past the volume)
            // and weighs it by 0
            const unsigned idx = __umul24(min((unsigned)h, (unsigned)nh), ntr) + __umul24(t, nr) + q;
            // kept in place (volatile) so the compiler neither sinks it to the end
            // of the step nor copies the loaded value
            asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(acc) : "v"(plen), "v"(pval));
            pval = Store<VT>::ldb(vol, idx);
            plen = q < 0 ? 0.0f : len;
        }
    } visit{vol, g.n_h, g.n_theta, g.n_r, g.n_theta * g.n_r, 0.0f, 0.0f, 0.0f};
    traverse<true, false, PRECISE, REFINE>(g, T, V, r, a0, a1, ih, it, ir, visit);
    return fmaf(visit.plen, visit.pval, visit.acc);
}

// Workgroup of 256 lanes (4 waves).  With nsplit pieces per ray the
// workgroup covers 256 / nsplit rays; wave w takes piece w % nsplit of the
// 64 rays of pixel group w / nsplit (an 8 x 8 tile), so the lanes of a wave
// walk the same stretch of neighbouring rays and their gathers stay coherent.
// Partial sums meet in LDS.  blockIdx.y = item of the launch (a scan and one of
// its views); blockIdx.x indexes that geometry's dispatch order (per-XCD row
// bands, centre-out columns); workgroups past the item's tile count exit.
template <int VT, int PT, bool SART>
__global__ __launch_bounds__(256) void fp_kernel(const FpLaunch L) {
    const FpItem &item = L.item[blockIdx.y];
    if ((int)blockIdx.x >= item.nwg) return;
    const GeomDev &g = item.g;
    const void *__restrict__ vol = item.vol;
    void *__restrict__ proj = item.proj;
    const void *__restrict__ pw = item.pw;
    float *__restrict__ rho = item.rho;
    const int pwt = item.pwt, nsplit = item.ns;
    extern __shared__ float2 smem[];
    const Tabs T = stage_tables(g, smem);
    float *part = (float *)(smem + table_floats2(g));
    __syncthreads();
    const int k = item.view;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int groups = 4 / nsplit;           // 8x8 pixel groups per workgroup
    const int piece = wave % nsplit, grp = wave / nsplit;
    // workgroup tile: 8 * groups wide, 8 high
    const int tw = 8 * groups;
    const int tiles_u = (g.cols + tw - 1) / tw;
    const int tile = g.fp_order[nsplit == 1 ? 0 : (nsplit == 2 ? 1 : 2)][blockIdx.x];
    const int u = (tile % tiles_u) * tw + grp * 8 + (lane & 7);
    const int v = (tile / tiles_u) * 8 + (lane >> 3);
    const bool live = u < g.cols && v < g.rows;
    const ViewDev &V = g.views[k];
    const Frame F = grid_frame(g);
    Ray r;
    double dx, dy, dz;
    ray_setup(g, V, live ? u : 0, live ? v : 0, F, r, dx, dy, dz);
    if (live && clip_support(g, T, r)) r.flags |= RAY_HIT;
    const __amdgpu_buffer_rsrc_t vrs =
        buffer_rsrc(vol, (unsigned)g.n_h * (unsigned)g.n_theta * (unsigned)g.n_r * (unsigned)Store<VT>::kSize);
    // rays whose reference point lies far from their closest approach (nearly
    // parallel to the axis) need the shell roots as small differences, and
    // rays passing near the axis may need FP64 edge crossings; wave-wide
    // choices
    const bool far_ref = (r.flags & RAY_HIT) && (r.k2 < 0.25f || fabsf(r.sc) > (float)g.r_max_d);
    float acc;
    if (__ballot(far_ref))
        acc = fp_piece<VT, true, true>(g, T, V, F, r, vrs, piece, nsplit);
    else if (__ballot(needs_refine(r, r.s_in, r.s_out)))
        acc = fp_piece<VT, false, true>(g, T, V, F, r, vrs, piece, nsplit);
    else
        acc = fp_piece<VT, false, false>(g, T, V, F, r, vrs, piece, nsplit);
    if (nsplit > 1) {
        part[threadIdx.x] = acc;
        __syncthreads();
        if (piece != 0) return;
        for (int p = 1; p < nsplit; ++p) acc += part[threadIdx.x + 64 * p];
    }
    const size_t j = ((size_t)k * g.rows + v) * g.cols + u;
    if (!SART) {
        // plain projection, or a difference from given projections (pw)
        if (live) Store<PT>::st(proj, j, pw ? ld_any(pw, pwt, j) - acc : acc);
        return;
    }
    float rj = 0.0f;
    if (live) {
        const float L = (r.flags & RAY_HIT) ? row_sum_fp64(g, V, dx, dy, dz) : 0.0f;
        const float pj = Store<PT>::ld(proj, j);
        const float w = pw ? ld_any(pw, pwt, j) : 1.0f;
        rj = (L > 0.0f) ? w * (pj - acc) / L : 0.0f;
        rho[(size_t)v * g.cols + u] = rj;
    }
    // the wave's 64 pixels are one aligned 8x8 tile: store its largest |rho|
    // (whole waves reach this point; a tile past the last column is skipped)
    const float tm = wave_max(fabsf(rj));
    const int tu = ((tile % tiles_u) * tw + grp * 8) >> 3;
    if (lane == 0 && tu * 8 < g.cols) item.tmax[(size_t)(tile / tiles_u) * ((g.cols + 7) >> 3) + tu] = tm;
}

// Exact traversal of every ray of one view, recording its pieces inside the
// grid (length > 0; the hole r < r_min is skipped).  Count pass (fill = 0):
// counts[pix] = pieces and rowsum[pix] = L_j (closed form, FP64).  Fill pass:
// the pieces of ray pix go to cells/lens from rowptr[pix], in walk order,
// never past rowptr[pix + 1].  One kernel for both passes, so both walk with
// the same instructions and find the same pieces.
__global__ __launch_bounds__(256) void record_kernel(GeomDev g, int view, int fill, const int32_t *__restrict__ rowptr,
                                                     int32_t *__restrict__ counts, int32_t *__restrict__ cells,
                                                     float *__restrict__ lens, float *__restrict__ rowsum) {
    extern __shared__ float2 smem[];
    const Tabs T = stage_tables(g, smem);
    __syncthreads();
    const int pix = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (pix >= g.rows * g.cols) return;
    const int u = pix % g.cols, v = pix / g.cols;
    const ViewDev &V = g.views[view];
    const Frame F = grid_frame(g);
    Ray r;
    double dx, dy, dz;
    ray_setup(g, V, u, v, F, r, dx, dy, dz);
    if (clip_support(g, T, r)) r.flags |= RAY_HIT;
    struct Record {
        int32_t *cells;
        float *lens;
        int nh, nt, nr, n, pos, cap;
        __device__ __forceinline__ void operator()(int h, int t, int q, float len) {
            // the walk may leave the grid by a step of rounding at its faces:
            // record only cells of the grid
            if (q < 0 || q >= nr || (unsigned)h >= (unsigned)nh || !(len > 0.0f)) return;
            if (n < cap) {
                cells[pos + n] = (h * nt + t) * nr + q;
                lens[pos + n] = len;
            }
            ++n;
        }
    } rec{cells, lens, g.n_h, g.n_theta, g.n_r, 0, fill ? rowptr[pix] : 0, fill ? rowptr[pix + 1] - rowptr[pix] : 0};
    if ((r.flags & RAY_HIT) && r.s_out > r.s_in) {
        int ih, it, ir;
        cell_at(g, r, F, r.s_in, ih, it, ir);
        traverse<true, false, true, true>(g, T, V, r, r.s_in, r.s_out, ih, it, ir, rec);
    }
    if (!fill) {
        counts[pix] = rec.n;
        rowsum[pix] = (r.flags & RAY_HIT) ? row_sum_fp64(g, V, dx, dy, dz) : 0.0f;
    } else {
        // a row the fill pass found shorter is padded with empty entries
        for (int i = rec.n; i < rec.cap; ++i) {
            cells[rec.pos + i] = 0;
            lens[rec.pos + i] = 0.0f;
        }
    }
}

__global__ __launch_bounds__(256) void rowsum_kernel(GeomDev g, float *__restrict__ out, int view_begin) {
    const int k = view_begin + blockIdx.y;
    const int tiles_u = (g.cols + 15) / 16;
    const int u = (blockIdx.x % tiles_u) * 16 + (threadIdx.x & 15);
    const int v = (blockIdx.x / tiles_u) * 16 + (threadIdx.x >> 4);
    if (u >= g.cols || v >= g.rows) return;
    const ViewDev &V = g.views[k];
    const double fu = (double)u, fv = (double)v;
    const double dx = fma(fv, V.V[0], fma(fu, V.U[0], V.d0[0]));
    const double dy = fma(fv, V.V[1], fma(fu, V.U[1], V.d0[1]));
    const double dz = fma(fv, V.V[2], fma(fu, V.U[2], V.d0[2]));
    out[((size_t)k * g.rows + v) * g.cols + u] = row_sum_fp64(g, V, dx, dy, dz);
}

// ------------------------------------------------------------ back-projection

// Projection of one bounding point of the block's convex hull
// slab x wedge x disc(r_B) in view V, for point index `pt` (two z levels per
// polygon corner; the polygon circumscribes the outer arc).  Points with
// pt >= count leave the box untouched.  Sets `behind` if the point is not in
// front of the source.
__device__ __forceinline__ void footprint_point(const GeomDev &g, const Tabs &T, const ViewDev &V, const Block &B,
                                                int pt, float &umin, float &umax, float &vmin, float &vmax,
                                                float &behind, float &lmin) {
    const float rO = T.r[B.rB].x * (1.0f + 1e-6f) + 1e-6f;
    const float rI = T.r[B.rA].x;
    const bool full = (B.tB - B.tA) >= g.n_theta;
    const int pi = pt >> 1;
    int npoly;
    float px = 0.0f, py = 0.0f;
    if (full) {
        npoly = 4;
        const float c = rO * 1.41421356f * (1.0f + 1e-6f);
        px = (pi == 0 || pi == 3) ? c : -c;
        py = (pi < 2) ? c : -c;
    } else {
        const float thA = g.theta0 + B.tA * g.dtheta;
        const float om = (B.tB - B.tA) * g.dtheta;
        const int nseg = max(1, (int)ceilf(om * (4.0f / 3.14159265f) - 1e-4f));
        const float del = om / nseg;
        // hardware sine/cosine (~1e-6 absolute): the polygon is inflated by 1e-5
        // and the pixel box keeps a 0.05-pixel margin, far above that error
        const float rc = rO / __cosf(0.5f * del) * (1.0f + 1e-5f);
        npoly = nseg + 3;
        if (pi <= nseg) {
            const float ang = thA + pi * del;
            px = rc * __cosf(ang);
            py = rc * __sinf(ang);
        } else {
            const float ang = (pi == nseg + 1) ? thA : thA + om;
            px = rI * __cosf(ang);
            py = rI * __sinf(ang);
        }
    }
    if (pi >= npoly) return;
    const float pz = (pt & 1) ? T.h[B.hB].x + 1e-5f : T.h[B.hA].x - 1e-5f;
    const float X = px - V.af[0], Y = py - V.af[1], Z = pz - V.af[2];
    const float lam = V.Qi[0] * X + V.Qi[1] * Y + V.Qi[2] * Z;
    const float uu = V.Qi[3] * X + V.Qi[4] * Y + V.Qi[5] * Z;
    const float vv = V.Qi[6] * X + V.Qi[7] * Y + V.Qi[8] * Z;
    if (lam > 1e-6f) {
        const float il = 1.0f / lam;
        lmin = fminf(lmin, lam);
        umin = fminf(umin, uu * il);
        umax = fmaxf(umax, uu * il);
        vmin = fminf(vmin, vv * il);
        vmax = fmaxf(vmax, vv * il);
    } else {
        behind = 1.0f;
    }
}

// Pixel index box from the projected extent (with a small margin, clipped to
// the detector).  Returns false if empty.
__device__ __forceinline__ bool footprint_box(const GeomDev &g, float umin, float umax, float vmin, float vmax,
                                              float behind, int &u0, int &u1, int &v0, int &v1) {
    if (behind > 0.0f) {
        u0 = 0;
        u1 = g.cols - 1;
        v0 = 0;
        v1 = g.rows - 1;
        return true;
    }
    const float m = 0.05f;
    const float fu0 = fmaxf(ceilf(umin - m), 0.0f), fu1 = fminf(floorf(umax + m), (float)(g.cols - 1));
    const float fv0 = fmaxf(ceilf(vmin - m), 0.0f), fv1 = fminf(floorf(vmax + m), (float)(g.rows - 1));
    if (!(fu1 >= fu0 && fv1 >= fv0)) return false;
    u0 = (int)fu0;
    u1 = (int)fu1;
    v0 = (int)fv0;
    v1 = (int)fv1;
    return true;
}

// Detector box of the block in view V; the whole wave participates (each lane
// projects one hull point, then min/max across the wave).  If cellrays is
// given, it receives a bound on the number of rays of the box that meet any
// one cell of diameter at most dcell: the box size, or fewer from the
// projection's scale.  With X' = X - a, u = (q_u X') / (q_l X') and
// v = (q_v X') / (q_l X') (q_* rows of Qi), so |du/dX| <= (|q_u| + |u| |q_l|) / lam
// with lam = q_l X'; over the block hull (a convex prism inside the projected
// polygon prism) |u| and 1/lam are largest at its vertices.  A cell's convex
// hull lies in the block hull, so its image spans at most ext_u = dcell
// max|du/dX| columns and ext_v rows, which hold at most
// (ext_u + 1)(ext_v + 1) pixel centres.
__device__ bool footprint(const GeomDev &g, const Tabs &T, const ViewDev &V, const Block &B, int &u0, int &u1,
                          int &v0, int &v1, float dcell = 0.0f, float *cellrays = nullptr) {
    float umin = CYL_INF, umax = -CYL_INF, vmin = CYL_INF, vmax = -CYL_INF, behind = 0.0f, lmin = CYL_INF;
    footprint_point(g, T, V, B, threadIdx.x & 63, umin, umax, vmin, vmax, behind, lmin);
    umin = wave_min(umin);
    umax = wave_max(umax);
    vmin = wave_min(vmin);
    vmax = wave_max(vmax);
    behind = wave_max(behind);
    const bool any = footprint_box(g, umin, umax, vmin, vmax, behind, u0, u1, v0, v1);
    if (cellrays && any) {
        float rays = (float)((u1 - u0 + 1) * (v1 - v0 + 1));
        if (!(behind > 0.0f)) {
            lmin = wave_min(lmin);
            const float ql = sqrtf(V.Qi[0] * V.Qi[0] + V.Qi[1] * V.Qi[1] + V.Qi[2] * V.Qi[2]);
            const float qu = sqrtf(V.Qi[3] * V.Qi[3] + V.Qi[4] * V.Qi[4] + V.Qi[5] * V.Qi[5]);
            const float qv = sqrtf(V.Qi[6] * V.Qi[6] + V.Qi[7] * V.Qi[7] + V.Qi[8] * V.Qi[8]);
            const float au = fmaxf(fabsf(umin), fabsf(umax)), av = fmaxf(fabsf(vmin), fabsf(vmax));
            const float eu = dcell * (qu + au * ql) / lmin * 1.001f;
            const float ev = dcell * (qv + av * ql) / lmin * 1.001f;
            rays = fminf(rays, (floorf(eu) + 1.0f) * (floorf(ev) + 1.0f));
        }
        *cellrays = rays;
    }
    return any;
}

// Accumulator slot of block-local cell (h, t, q): rows of wr + 1 words (the
// last a spare), planes of wt + 2 rows (the first and last spare) plus one
// word, odd strides so neighbouring cells in theta and h fall in different LDS
// banks.  A walk that steps one cell past the block's theta faces or its
// radial faces (rounding at a face) lands in a spare word; one past its h
// faces lands below 0 or at or above block_slots - 1, where the scatter
// clamps it to the last word, a spare too.
__device__ __forceinline__ int slot_rs(const Block &B) { return (B.rB - B.rA) + 1; }
__device__ __forceinline__ int slot_ps(const Block &B) { return (B.tB - B.tA + 2) * slot_rs(B) + 1; }
__device__ __forceinline__ int slot(const Block &B, int h, int t, int q) {
    return h * slot_ps(B) + (t + 1) * slot_rs(B) + q;
}

__device__ __forceinline__ int block_slots(const Block &B) { return (B.hB - B.hA) * slot_ps(B) + 1; }

// Trace ray (u, v) of view V through block B (a block or a super-block) and
// add its lengths into one 64-bit fixed-point accumulator per cell,
// acc64 = c 2^32 + n with c = sum rint(t_jm y_j cscale) and
// n = sum rint(t_jm nscale): one integer LDS atomic per step, and integer sums
// do not depend on their order.  The scales keep |c| and n below 2^31 (see
// sart_scales), so the low word never carries into the high word; yj is
// y_j cscale, and nscale = 0 accumulates c alone.
__device__ __forceinline__ void bp_ray(const GeomDev &g, const Tabs &T, const Frame &F, const ViewDev &V,
                                       const Block &B, int u, int v, float yj, unsigned long long *acc64,
                                       float nscale) {
    // slot of cell (h, t, q) = h ps + t rs + q - (hA ps + (tA - 1) rs + rA)
    // (see slot), clamped into the accumulator
    const int rs = slot_rs(B), ps = slot_ps(B);
    const int off = B.hA * ps + (B.tA - 1) * rs + B.rA;
    struct Scatter {
        unsigned long long *b64;
        int ps, rs, off, last;
        float yj, nscale;
        __device__ __forceinline__ void operator()(int h, int t, int q, float len) {
            const unsigned loc = min((unsigned)((int)(__umul24(h, ps) + __umul24(t, rs)) + q - off), (unsigned)last);
            const unsigned int c = (unsigned int)round_half_up(len * yj);
            const unsigned int n = (unsigned int)round_half_up(len * nscale);
            atomicAdd(&b64[loc], ((unsigned long long)c << 32) | n);
        }
    } visit{acc64, ps, rs, off, block_slots(B) - 1, yj, nscale};
    walk_block_ray(g, T, F, V, B, u, v, visit);
}

// Bound on the length of a ray inside one cell of block B (the cell's
// diameter, with the outer radius of the block for the arc), inflated by 1e-3.
__device__ __forceinline__ float cell_diameter(const GeomDev &g, const Tabs &T, const Block &B) {
    const float rB = T.r[B.rB].x;
    const float dxy = g.dtheta >= 3.14159265f
                          ? 2.0f * rB
                          : sqrtf(g.dr * g.dr + 4.0f * rB * rB * sinf(0.5f * g.dtheta) * sinf(0.5f * g.dtheta));
    return sqrtf(g.dh * g.dh + dxy * dxy) * 1.001f;
}

// Fixed-point scales of a super-block's SART update, {nscale, 1/nscale,
// cscale, 1/cscale}, computed by one wave.  With D the cell diameter (a bound
// on any chord through one cell), R_k the bound on the rays of view k that
// meet one cell (footprint) and m_k the largest |rho| over the 8x8 tiles that
// cover view k's footprint box (the residual FP's tile maxima; at least the
// largest |rho| of the footprint), n_m <= D sum_k R_k and |c_m| <= D sum_k R_k m_k; the scales are the powers
// of two that keep these bounds at or below 2^30.  Each term is rounded by at
// most 1/2, and a cell's sum has at most 2^30 terms (at most 2^28 pixels per
// update, the host's limit, and at most 4 pieces of a ray in one cell), so
// the sums of one cell stay below 1.5 2^30: c fits the signed high word of
// acc64 and n never carries out of the low word.
__device__ float4 sart_scales(const GeomDev &g, const Tabs &T, const Block &B, const float *__restrict__ rho,
                              const int32_t *__restrict__ vlist, int view_begin, int view_end) {
    const int lane = threadIdx.x & 63;
    const float dcell = cell_diameter(g, T, B);
    const size_t npv = (size_t)g.rows * g.cols;
    float nb = 0.0f, cb = 0.0f;
    for (int k = view_begin; k < view_end; ++k) {
        const int view = vlist ? vlist[k] : k;
        float rays;
        int u0, u1, v0, v1;
        if (!footprint(g, T, g.views[view], B, u0, u1, v0, v1, dcell, &rays)) continue;
        u0 = __builtin_amdgcn_readfirstlane(u0);
        u1 = __builtin_amdgcn_readfirstlane(u1);
        v0 = __builtin_amdgcn_readfirstlane(v0);
        v1 = __builtin_amdgcn_readfirstlane(v1);
        // largest |rho| of the aligned 8x8 tiles that cover the box
        const float *tk = rho + (size_t)(view_end - view_begin) * npv + (size_t)(k - view_begin) * tile_count(g);
        const int tpu = (g.cols + 7) >> 3, tu0 = u0 >> 3, tv0 = v0 >> 3;
        const int ntu = (u1 >> 3) - tu0 + 1, nt = ntu * ((v1 >> 3) - tv0 + 1);
        float rmax = 0.0f;
        for (int p = lane; p < nt; p += 64) rmax = fmaxf(rmax, tk[(size_t)(tv0 + p / ntu) * tpu + tu0 + p % ntu]);
        rmax = wave_max(rmax);
        nb += rays;
        cb = fmaf(rays, rmax, cb);
    }
    float4 sc = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    if (nb > 0.0f) {
        int e;
        frexpf(1073741824.0f / (dcell * nb), &e);
        sc.x = ldexpf(1.0f, e - 1);
        sc.y = ldexpf(1.0f, 1 - e);
        if (cb > 0.0f) {
            frexpf(1073741824.0f / (dcell * cb), &e);
            sc.z = ldexpf(1.0f, e - 1);
            sc.w = ldexpf(1.0f, 1 - e);
        }
    }
    return sc;
}

// Fixed-point scale of a super-block's plain transpose, {cscale, 1/cscale},
// computed by one wave: |c_m| <= D sum_k R_k m_k as for sart_scales, with
// m_k the largest |y| over view k's footprint box (read pixel by pixel: the
// caller's projections carry no tile maxima).
template <int PT>
__device__ float2 plain_scales(const GeomDev &g, const Tabs &T, const Block &B, const void *__restrict__ y,
                               int view_begin, int view_end) {
    const int lane = threadIdx.x & 63;
    const float dcell = cell_diameter(g, T, B);
    float cb = 0.0f;
    for (int k = view_begin; k < view_end; ++k) {
        float rays;
        int u0, u1, v0, v1;
        if (!footprint(g, T, g.views[k], B, u0, u1, v0, v1, dcell, &rays)) continue;
        u0 = __builtin_amdgcn_readfirstlane(u0);
        u1 = __builtin_amdgcn_readfirstlane(u1);
        v0 = __builtin_amdgcn_readfirstlane(v0);
        v1 = __builtin_amdgcn_readfirstlane(v1);
        const int nu = u1 - u0 + 1, npix = nu * (v1 - v0 + 1);
        const size_t vb = (size_t)k * g.rows;
        float ymax = 0.0f;
        for (int p = lane; p < npix; p += 64)
            ymax = fmaxf(ymax, fabsf(Store<PT>::ld(y, (vb + v0 + p / nu) * g.cols + u0 + p % nu)));
        cb = fmaf(rays, wave_max(ymax), cb);
    }
    float2 sc = make_float2(1.0f, 1.0f);
    if (cb > 0.0f) {
        int e;
        frexpf(1073741824.0f / (dcell * cb), &e);
        sc.x = ldexpf(1.0f, e - 1);
        sc.y = ldexpf(1.0f, 1 - e);
    }
    return sc;
}

// Back-projection on super-blocks.  With integer sums the order of the
// additions does not matter, so the 4 waves of a workgroup share one
// accumulator for a super-block, and a ray that crosses several of its
// blocks is set up once.  The waves take batches of 64
// footprint pixels from an LDS counter that runs across the views of the
// call: each wave walks the views in the same order and computes the same
// footprints (same code, same inputs), and so finds the same batch boundaries
// without synchronising.  Wave 0 alone finds the fixed-point scales.
// SART: y holds the FP32 residual images of the update's positions (then
// their tile maxima), each cell accumulates (c, n) and
// vol += lam * wv * c / n where n > 0.  Plain transpose: y holds the caller's
// projections (type PT, [n_views][rows][cols]), each cell accumulates c alone
// (n scale 0) and vol = (accumulate ? vol : 0) + c for every cell.
// The walks run in the super-block's frame (block_frame).
template <int VT, int PT, bool SART, int SBB>
__device__ __forceinline__ void superblock_bp(const BpLaunch &L) {
    const BpItem &item = L.item[blockIdx.y];
    if ((int)blockIdx.x >= item.nwg) return;
    const GeomDev &g = item.g;
    const float *__restrict__ rho = (const float *)item.y;
    void *__restrict__ vol = item.vol;
    const void *__restrict__ vw = item.vw;
    const int view_begin = item.view_begin, view_end = item.view_end;
    const int accumulate = item.flags & 1, nonneg = (item.flags >> 1) & 1, vwt = item.flags >> 8;
    const float lam = item.lam;
    const int32_t *__restrict__ vlist = item.views;
    extern __shared__ float2 smem[];
    Tabs T;
    const int lane = threadIdx.x & 63;
    // super-blocks: outer rings first (their blocks carry the most work)
    constexpr int nthr = 64 * SBB;
    const SbShape sb = sb_shape(g, SBB);
    const int per_ring = sb.nst * sb.nsh;
    const int isr = sb.nsr - 1 - (int)blockIdx.x / per_ring;
    const int rem = (int)blockIdx.x % per_ring;
    const int ish = rem % sb.nsh, ist = rem / sb.nsh;
    Block B;
    B.hA = ish * sb.fh * g.bh;
    B.hB = min(B.hA + sb.fh * g.bh, g.n_h);
    B.tA = ist * sb.ft * g.bt;
    B.tB = min(B.tA + sb.ft * g.bt, g.n_theta);
    B.rA = isr * sb.fr * g.br;
    B.rB = min(B.rA + sb.fr * g.br, g.n_r);
    const int wt = B.tB - B.tA, wr = B.rB - B.rA;
    const int ncell = (B.hB - B.hA) * wt * wr;
    // the walks are boxed to the super-block, so they read its sector edges
    // (and one either side) only; then the accumulator words
    int mfr;
    const Frame F = block_frame(g, B, mfr);
    const int nedge = B.tB - B.tA + 3;
    for (int j = threadIdx.x; j < nedge; j += nthr) smem[j] = block_edge(g, B, mfr, j);
    T.r = g.r_tab;
    T.h = g.h_tab;
    T.cs = smem;
    T.cs_lo = B.tA - 1;
    T.cs_n = nedge - 1;
    unsigned long long *acc64 = (unsigned long long *)(smem + sb_edge_words(g, sb));
    // The allocation (bp_lds_bytes) holds the block_slots of a full-size
    // super-block and 4 words more: word nslot holds the batch counter, the
    // next two the fixed-point scales.
    const int nslot = block_slots(B);
    unsigned int *counter = (unsigned int *)(acc64 + nslot);
    float *scales = (float *)(acc64 + nslot + 1);
    for (int i = threadIdx.x; i < nslot; i += nthr) acc64[i] = 0ull;
    if (threadIdx.x == 0) *counter = 0u;
    const size_t npv = (size_t)g.rows * g.cols;
    // wave 0 finds the fixed-point scales and shares them through LDS
    if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0) {
        float4 sc;
        if (SART) {
            sc = sart_scales(g, T, B, rho, vlist, view_begin, view_end);
        } else {
            const float2 c = plain_scales<PT>(g, T, B, item.y, view_begin, view_end);
            sc = make_float4(0.0f, 0.0f, c.x, c.y);
        }
        if (lane == 0) {
            scales[0] = sc.x;
            scales[1] = sc.y;
            scales[2] = sc.z;
            scales[3] = sc.w;
        }
    }
    __syncthreads();
    const float nscale = scales[0], inv_nscale = scales[1], cscale = scales[2], inv_cscale = scales[3];
    // batches of 64 pixels, views in order: view k owns batch numbers
    // [first, first + nbatch_k)
    int k = view_begin, first = 0, nbatch = -1, u0 = 0, v0 = 0, nu = 1, npix = 0;
    for (;;) {
        unsigned int bi = 0;
        if (lane == 0) bi = atomicAdd(counter, 1u);
        const int b = (int)__builtin_amdgcn_readfirstlane(bi);
        // advance to the view holding batch b
        while (k < view_end && (nbatch < 0 || b >= first + nbatch)) {
            if (nbatch >= 0) {
                first += nbatch;
                ++k;
                nbatch = -1;
                continue;
            }
            const int view = vlist ? vlist[k] : k;
            int uu0, uu1, vv0, vv1;
            if (footprint(g, T, g.views[view], B, uu0, uu1, vv0, vv1)) {
                u0 = __builtin_amdgcn_readfirstlane(uu0);
                v0 = __builtin_amdgcn_readfirstlane(vv0);
                nu = __builtin_amdgcn_readfirstlane(uu1) - u0 + 1;
                npix = nu * (__builtin_amdgcn_readfirstlane(vv1) - v0 + 1);
                nbatch = (npix + 63) / 64;
            } else {
                nbatch = 0;
            }
        }
        if (k >= view_end) break;
        const int p = (b - first) * 64 + lane;
        if (p < npix) {
            const int view = vlist ? vlist[k] : k;
            const int v = v0 + p / nu;
            const int u = u0 + p % nu;
            const float yj = SART ? rho[(size_t)(k - view_begin) * npv + (size_t)v * g.cols + u]
                                  : Store<PT>::ld(item.y, (size_t)k * npv + (size_t)v * g.cols + u);
            if (SART || yj != 0.0f)
                bp_ray(g, T, F, g.views[view], B, u, v, yj * cscale, acc64, nscale);
        }
    }
    __syncthreads();
    // update: nthr lanes over the cells, i = (h wt + t) wr + q stepped by nthr
    const int dq = nthr % wr, dt = (nthr / wr) % wt, dh = nthr / (wr * wt);
    const int i0 = (int)threadIdx.x;
    int q = i0 % wr, t = (i0 / wr) % wt, h = i0 / (wr * wt);
    for (int i = i0; i < ncell; i += nthr) {
        if (i != i0) {
            q += dq;
            const int c1 = q >= wr ? 1 : 0;
            q -= c1 ? wr : 0;
            t += dt + c1;
            const int c2 = t >= wt ? 1 : 0;
            t -= c2 ? wt : 0;
            h += dh + c2;
        }
        const unsigned long long a = acc64[slot(B, h, t, q)];
        if (!SART) {
            const size_t gi = ((size_t)(B.hA + h) * g.n_theta + (B.tA + t)) * g.n_r + (B.rA + q);
            const float c = (float)(int)(unsigned int)(a >> 32) * inv_cscale;
            Store<VT>::st(vol, gi, (accumulate ? Store<VT>::ld(vol, gi) : 0.0f) + c);
            continue;
        }
        const float n = (float)(unsigned int)a * inv_nscale;
        if (n > 0.0f) {
            const size_t gi = ((size_t)(B.hA + h) * g.n_theta + (B.tA + t)) * g.n_r + (B.rA + q);
            const float c = (float)(int)(unsigned int)(a >> 32) * inv_cscale;
            const float w = vw ? ld_any(vw, vwt, gi) : 1.0f;
            float m = Store<VT>::ld(vol, gi) + lam * w * c * frcp(n);
            if (nonneg && m < 0.0f) m = 0.0f;
            Store<VT>::st(vol, gi, m);
        }
    }
}

// SART update (Eq. 7 over the update's views) on super-blocks.
template <int VT, int SBB>
__global__ __launch_bounds__(64 * SBB, 4) void sart_bp_kernel(const BpLaunch L) {
    superblock_bp<VT, CYL_F32, true, SBB>(L);
}

// Plain transpose A^T y over views [view_begin, view_end) on super-blocks.
template <int VT, int PT, int SBB>
__global__ __launch_bounds__(64 * SBB, 4) void bp_kernel(const BpLaunch L) {
    superblock_bp<VT, PT, false, SBB>(L);
}

// ------------------------------------------------------------ elementwise

// out = a + b over n values (storage types at, bt, ot), FP32 arithmetic.
template <int OT>
__global__ __launch_bounds__(256) void add_kernel(size_t n, const void *__restrict__ a, int at,
                                                  const void *__restrict__ b, int bt, void *__restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        Store<OT>::st(out, i, ld_any(a, at, i) + ld_any(b, bt, i));
}

// ------------------------------------------------------------ launchers

static int launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return CYL_EDEVICE;
    }
    return CYL_OK;
}

static size_t table_bytes(const GeomDev &g) {
    return sizeof(float2) * ((size_t)(g.n_r + 1) + (g.n_h + 1) + (g.n_theta + 1));
}

int launch_record(const cyl_geom *G, int view, const int32_t *rowptr, int32_t *counts, int32_t *cells, float *lens,
                  float *rowsum, hipStream_t st) {
    const GeomDev &g = G->dev;
    const dim3 grid((unsigned)((g.rows * g.cols + 255) / 256));
    const size_t lds = table_bytes(g);
    hipLaunchKernelGGL(record_kernel, grid, dim3(256), lds, st, g, view, cells ? 1 : 0, rowptr, counts, cells, lens,
                       rowsum);
    return launch_check("record");
}

// LDS of a super-block launch: the super-block's sector edges, then the
// 64-bit accumulator words of its largest super-block (block_slots of
// fh bh slabs, ft bt sectors and fr br rings), its batch counter and two
// scale words, and one word to spare.
static size_t bp_lds_bytes(const GeomDev &g, int sbb) {
    const SbShape sb = sb_shape(g, sbb);
    const size_t slots = (size_t)(sb.fh * g.bh) * ((size_t)(sb.ft * g.bt + 2) * (sb.fr * g.br + 1) + 1) + 1;
    return sizeof(float2) * (size_t)sb_edge_words(g, sb) + sizeof(unsigned long long) * (slots + 4);
}

// Blocks per super-block of a grid: 8 when the grid has at most 2^25 cells
// and still gives at least 8 super-blocks per CU (2048); else 4.  Measured per
// view: 8 took the 256x720x128 update (2944 super-blocks) from 0.403 to 0.388
// ms, unposed and posed alike; 4 kept the 512x1440x256 posed one at 3.05 ms
// against 3.61 and the 32x512x256 one (512 super-blocks) at 0.295 against
// 0.333.  A property of the grid alone, so a scan's result does not depend on
// the batch it is launched with; a launch holds items of one size.
static int grid_sbb(const GeomDev &g) {
    if ((int64_t)g.n_h * g.n_theta * g.n_r > ((int64_t)1 << 25)) return 4;
    const SbShape sb = sb_shape(g, 8);
    return (int64_t)sb.nsh * sb.nst * sb.nsr >= 2048 ? 8 : 4;
}

// Rays per item below which each ray is split over neighbouring lanes so one
// view still fills the GPU.  Chosen per item, so an item's result does not
// depend on what else shares its launch.
static int fp_split(const GeomDev &g, int nv) {
    const long rays = (long)g.rows * g.cols * nv;
    if (rays >= (4L << 20)) return 1;
    if (rays >= (1L << 20)) return 2;
    return 4;
}

static FpItem fp_item(const cyl_geom *G, const void *vol, void *proj, int view, int ns, const void *pw, int pwt,
                      float *rho, float *tmax = nullptr) {
    const GeomDev &g = G->dev;
    const int tw = 8 * (4 / ns);
    FpItem it;
    it.g = G->dev;
    it.vol = vol;
    it.proj = proj;
    it.pw = pw;
    it.rho = rho;
    it.tmax = tmax;
    it.view = view;
    it.ns = ns;
    it.nwg = ((g.cols + tw - 1) / tw) * ((g.rows + 7) / 8);
    it.pwt = pwt;
    return it;
}

// One back-projection item; its workgroup count is set by launch_bp_batch,
// which picks the super-block size.
static BpItem bp_item(const cyl_geom *G, const void *y, int vb, int ve, void *vol, int accumulate, const void *vw,
                      int vwt, float lam, int nonneg, const int32_t *views = nullptr) {
    BpItem it;
    it.g = G->dev;
    it.y = y;
    it.vol = vol;
    it.vw = vw;
    it.views = views;
    it.view_begin = vb;
    it.view_end = ve;
    it.nwg = 0;
    it.flags = (accumulate ? 1 : 0) | (nonneg ? 2 : 0) | (vwt << 8);
    it.lam = lam;
    return it;
}

// Launch sizes of a batch: the widest item sets grid.x, the largest tables set
// the LDS.
struct LaunchShape {
    int maxwg = 0;
    size_t lds = 0;
    int sbb = 4;        // BP: blocks per super-block (and waves per workgroup)
};

template <int VT, int PT>
static void launch_fp_t(const FpLaunch &L, const LaunchShape &sh, bool sart, hipStream_t st) {
    dim3 grid(sh.maxwg, L.n);
    if (sart)
        hipLaunchKernelGGL((fp_kernel<VT, PT, true>), grid, dim3(256), sh.lds, st, L);
    else
        hipLaunchKernelGGL((fp_kernel<VT, PT, false>), grid, dim3(256), sh.lds, st, L);
}

template <int VT>
static void launch_fp_v(const FpLaunch &L, const LaunchShape &sh, int pt, bool sart, hipStream_t st) {
    switch (pt) {
        case CYL_F32: launch_fp_t<VT, CYL_F32>(L, sh, sart, st); break;
        case CYL_F16: launch_fp_t<VT, CYL_F16>(L, sh, sart, st); break;
        default: launch_fp_t<VT, CYL_BF16>(L, sh, sart, st); break;
    }
}

// Launches a filled FpLaunch (1 <= L.n <= kMaxBatch); geoms[i] is item i's geometry.
static void launch_fp_batch(const FpLaunch &L, const cyl_geom *const *geoms, int vt, int pt, bool sart,
                            hipStream_t st) {
    LaunchShape sh;
    for (int i = 0; i < L.n; ++i) {
        sh.maxwg = std::max(sh.maxwg, L.item[i].nwg);
        sh.lds = std::max(sh.lds, table_bytes(geoms[i]->dev) + 256 * sizeof(float));
    }
    switch (vt) {
        case CYL_F32: launch_fp_v<CYL_F32>(L, sh, pt, sart, st); break;
        case CYL_F16: launch_fp_v<CYL_F16>(L, sh, pt, sart, st); break;
        default: launch_fp_v<CYL_BF16>(L, sh, pt, sart, st); break;
    }
}

// Plain or SART FP of views [vb, vb + nv) of one scan, kMaxBatch views per launch.
static void launch_fp(const cyl_geom *G, const void *vol, int vt, void *proj, int pt, int vb, int nv, bool sart,
                      const void *pw, int pwt, float *rho, hipStream_t st) {
    const int ns = fp_split(G->dev, nv);
    const size_t npv = (size_t)G->rows * G->cols;
    const cyl_geom *geoms[kMaxBatch];
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        FpLaunch L;
        L.n = std::min(kMaxBatch, nv - v0);
        for (int i = 0; i < L.n; ++i) {
            L.item[i] = fp_item(G, vol, proj, vb + v0 + i, ns, pw, pwt, rho, sart ? rho + npv : nullptr);
            geoms[i] = G;
        }
        launch_fp_batch(L, geoms, vt, pt, sart, st);
    }
}

// SART residuals of the views views[0 .. nv) (host list) of one scan, all from
// the same volume; the residual image of views[i] goes to rho + i rows cols,
// its 8x8 tile maxima to rho + nv rows cols + i tile_count.
static void launch_fp_views(const cyl_geom *G, const void *vol, int vt, void *proj, int pt, const int32_t *views,
                            int nv, const void *pw, int pwt, float *rho, hipStream_t st) {
    const int ns = fp_split(G->dev, nv);
    const size_t npv = (size_t)G->rows * G->cols;
    const cyl_geom *geoms[kMaxBatch];
    for (int v0 = 0; v0 < nv; v0 += kMaxBatch) {
        FpLaunch L;
        L.n = std::min(kMaxBatch, nv - v0);
        for (int i = 0; i < L.n; ++i) {
            L.item[i] = fp_item(G, vol, proj, views[v0 + i], ns, pw, pwt, rho + (size_t)(v0 + i) * npv,
                                rho + (size_t)nv * npv + (size_t)(v0 + i) * tile_count(G->dev));
            geoms[i] = G;
        }
        launch_fp_batch(L, geoms, vt, pt, true, st);
    }
}

// Writes a host list of int32 into device memory through kernel arguments
// (stream-ordered, and the host list need not outlive the call).
struct I32Chunk {
    int32_t v[512];
};
__global__ __launch_bounds__(512) void store_i32_kernel(int32_t *__restrict__ dst, int n, const I32Chunk c) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.v[i];
}

static void store_i32(int32_t *dst, const int32_t *src, int n, hipStream_t st) {
    for (int i0 = 0; i0 < n; i0 += 512) {
        I32Chunk c;
        const int m = std::min(512, n - i0);
        for (int i = 0; i < m; ++i) c.v[i] = src[i0 + i];
        hipLaunchKernelGGL(store_i32_kernel, dim3(1), dim3(512), 0, st, dst + i0, m, c);
    }
}

template <int VT, int PT>
static void launch_bp_t(const BpLaunch &L, const LaunchShape &sh, bool sart, hipStream_t st) {
    dim3 grid(sh.maxwg, L.n);
#define CYL_BP_LAUNCH(SBB)                                                                      \
    do {                                                                                        \
        if (sart)                                                                               \
            hipLaunchKernelGGL((sart_bp_kernel<VT, SBB>), grid, dim3(64 * SBB), sh.lds, st, L); \
        else                                                                                    \
            hipLaunchKernelGGL((bp_kernel<VT, PT, SBB>), grid, dim3(64 * SBB), sh.lds, st, L);  \
    } while (0)
    if (sh.sbb == 8)
        CYL_BP_LAUNCH(8);
    else
        CYL_BP_LAUNCH(4);
#undef CYL_BP_LAUNCH
}

template <int VT>
static void launch_bp_v(const BpLaunch &L, const LaunchShape &sh, int pt, bool sart, hipStream_t st) {
    if (sart) {  // the SART update reads FP32 residuals, not the projections
        launch_bp_t<VT, CYL_F32>(L, sh, sart, st);
        return;
    }
    switch (pt) {
        case CYL_F32: launch_bp_t<VT, CYL_F32>(L, sh, sart, st); break;
        case CYL_F16: launch_bp_t<VT, CYL_F16>(L, sh, sart, st); break;
        default: launch_bp_t<VT, CYL_BF16>(L, sh, sart, st); break;
    }
}

static void launch_bp_batch(const BpLaunch &L, const cyl_geom *const *geoms, int vt, int pt, bool sart,
                            hipStream_t st) {
    for (int sbb = 8; sbb >= 4; sbb /= 2) {  // one launch per super-block size
        LaunchShape sh;
        sh.sbb = sbb;
        BpLaunch L2;
        L2.n = 0;
        const cyl_geom *g2[kMaxBatch];
        for (int i = 0; i < L.n; ++i) {
            if (grid_sbb(geoms[i]->dev) != sbb) continue;
            BpItem it = L.item[i];
            const SbShape sb = sb_shape(it.g, sbb);
            it.nwg = sb.nsr * sb.nst * sb.nsh;
            g2[L2.n] = geoms[i];
            L2.item[L2.n++] = it;
            sh.maxwg = std::max(sh.maxwg, it.nwg);
        }
        if (L2.n == 0) continue;
        for (int i = 0; i < L2.n; ++i) sh.lds = std::max(sh.lds, bp_lds_bytes(g2[i]->dev, sbb));
        switch (vt) {
            case CYL_F32: launch_bp_v<CYL_F32>(L2, sh, pt, sart, st); break;
            case CYL_F16: launch_bp_v<CYL_F16>(L2, sh, pt, sart, st); break;
            default: launch_bp_v<CYL_BF16>(L2, sh, pt, sart, st); break;
        }
    }
}

// Plain BP of views [vb, ve) (one item: the views accumulate in LDS) or the
// SART update of positions [vb, ve) (views[k], or view k without a list; the
// residual image of position k at rho + (k - vb) rows cols).
static void launch_bp(const cyl_geom *G, const void *y, int pt, int vb, int ve, void *vol, int vt, int accumulate,
                      bool sart, const float *rho, const void *vw, int vwt, float lam, int nonneg, hipStream_t st,
                      const int32_t *views = nullptr) {
    BpLaunch L;
    L.n = 1;
    L.item[0] = bp_item(G, sart ? (const void *)rho : y, vb, ve, vol, accumulate, vw, vwt, lam, nonneg, views);
    const cyl_geom *geoms[1] = {G};
    launch_bp_batch(L, geoms, vt, pt, sart, st);
}

// Makes the geometry's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        hipGetDevice(&prev);
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

static int check_range(const cyl_geom *G, int32_t vb, int32_t ve, const char *what) {
    if (vb < 0 || ve < vb || ve > G->n_views) {
        set_error("%s: view range [%d, %d) outside [0, %d)", what, vb, ve, G->n_views);
        return CYL_EINVAL;
    }
    return CYL_OK;
}

}  // namespace cyl

using namespace cyl;

extern "C" int cyl_fp(const cyl_geom *G, const void *vol, cyl_dtype vt, void *proj, cyl_dtype pt,
                      int32_t view_begin, int32_t view_end, void *hip_stream) {
    if (!G || !vol || !proj) {
        set_error("cyl_fp: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_fp volume")) || (rc = check_dtype(pt, "cyl_fp projections")) ||
        (rc = check_range(G, view_begin, view_end, "cyl_fp")))
        return rc;
    if (view_end == view_begin) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_fp: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_fp(G, vol, vt, proj, pt, view_begin, view_end - view_begin, false, nullptr, 0, nullptr,
              (hipStream_t)hip_stream);
    return launch_check("cyl_fp");
}

extern "C" int cyl_bp(const cyl_geom *G, const void *proj, cyl_dtype pt, void *vol, cyl_dtype vt,
                      int32_t view_begin, int32_t view_end, int32_t accumulate, void *hip_stream) {
    if (!G || !vol || !proj) {
        set_error("cyl_bp: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_bp volume")) || (rc = check_dtype(pt, "cyl_bp projections")) ||
        (rc = check_range(G, view_begin, view_end, "cyl_bp")))
        return rc;
    if (view_end == view_begin && accumulate) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_bp: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_bp(G, proj, pt, view_begin, view_end, vol, vt, accumulate ? 1 : 0, false, nullptr, nullptr, 0, 0.0f, 0,
              (hipStream_t)hip_stream);
    return launch_check("cyl_bp");
}

extern "C" int cyl_row_sums(const cyl_geom *G, float *out, int32_t view_begin, int32_t view_end,
                            void *hip_stream) {
    if (!G || !out) {
        set_error("cyl_row_sums: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_range(G, view_begin, view_end, "cyl_row_sums"))) return rc;
    if (view_end == view_begin) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_row_sums: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    const GeomDev &g = G->dev;
    dim3 grid(((g.cols + 15) / 16) * ((g.rows + 15) / 16), view_end - view_begin);
    hipLaunchKernelGGL(rowsum_kernel, grid, dim3(256), 0, (hipStream_t)hip_stream, g, out, view_begin);
    return launch_check("cyl_row_sums");
}

extern "C" size_t cyl_sart_workspace_bytes(const cyl_geom *G, const cyl_sart_params *) {
    if (!G) return 0;
    size_t n = ((size_t)G->rows * G->cols + tile_count(G->dev)) * sizeof(float);
    return (n + 255) & ~(size_t)255;
}

// Checks shared by the SART sweeps; `who` names the entry point in errors.
static int sart_check(const char *who, const cyl_geom *G, const cyl_sart_params *P, const void *proj, cyl_dtype pt,
                      const void *pw, cyl_dtype pwt, const void *vw, cyl_dtype vwt, const void *vol, cyl_dtype vt) {
    if (!G || !P || !proj || !vol) {
        set_error("%s: NULL argument", who);
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "SART volume")) || (rc = check_dtype(pt, "SART projections"))) return rc;
    if (pw && (rc = check_dtype(pwt, "SART projection weights"))) return rc;
    if (vw && (rc = check_dtype(vwt, "SART voxel weights"))) return rc;
    if (P->n_iter < 0 || P->start_iter < 0 || P->start_view < 0 || P->start_view > G->n_views) {
        set_error("%s: invalid iteration counts (n_iter %d, start %d/%d)", who, P->n_iter, P->start_iter,
                  P->start_view);
        return CYL_EINVAL;
    }
    if (!std::isfinite(P->lambda)) {
        set_error("%s: lambda must be finite", who);
        return CYL_EINVAL;
    }
    if (P->view_order)
        for (int i = 0; i < G->n_views; ++i)
            if (P->view_order[i] < 0 || P->view_order[i] >= G->n_views) {
                set_error("%s: view_order[%d] = %d out of range", who, i, P->view_order[i]);
                return CYL_EINVAL;
            }
    return CYL_OK;
}

// One sequential SART sweep (Eq. 7, one view per update) with its residual
// image and tile maxima at rho; the caller has validated the arguments.
static int sart_sweep(const cyl_geom *G, const cyl_sart_params *P, const void *proj, cyl_dtype pt, const void *pw,
                      cyl_dtype pwt, const void *vw, cyl_dtype vwt, void *vol, cyl_dtype vt, float *rho,
                      hipStream_t st, const char *who) {
    const float lam = (float)P->lambda;
    for (int it = P->start_iter; it < P->n_iter; ++it) {
        const int kv0 = (it == P->start_iter) ? P->start_view : 0;
        for (int kk = kv0; kk < G->n_views; ++kk) {
            const int k = P->view_order ? P->view_order[kk] : kk;
            launch_fp(G, vol, vt, const_cast<void *>(proj), pt, k, 1, true, pw, pwt, rho, st);
            launch_bp(G, nullptr, CYL_F32, k, k + 1, vol, vt, 0, true, rho, vw, vwt, lam, P->nonneg, st);
        }
        const int rc = launch_check(who);
        if (rc) return rc;
    }
    return CYL_OK;
}

extern "C" int cyl_sart_run(const cyl_geom *G, const cyl_sart_params *P, const void *proj, cyl_dtype pt,
                            const void *pw, cyl_dtype pwt, const void *vw, cyl_dtype vwt, void *vol,
                            cyl_dtype vt, void *workspace, size_t ws_bytes, void *hip_stream) {
    int rc;
    if ((rc = sart_check("cyl_sart_run", G, P, proj, pt, pw, pwt, vw, vwt, vol, vt))) return rc;
    const size_t need = cyl_sart_workspace_bytes(G, P);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_sart_run: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    if (P->start_iter >= P->n_iter) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sart_run: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    return sart_sweep(G, P, proj, pt, pw, pwt, vw, vwt, vol, vt, (float *)workspace, (hipStream_t)hip_stream,
                      "cyl_sart_run");
}

// Static scratch of cyl_sart_run_static: one copy per GPU, alive until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device array: host code uses only the address hipGetSymbolAddress returns
// for the current device (scratch_ptr), looked up once per device.
static __device__ __align__(256) unsigned char scratch[CYL_SART_STATIC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static void *scratch_dev[kMaxDevices];

// Device address of `scratch` on `device` (which must be current); null on
// failure, with the error set.
static void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("cyl_sart_run_static: device %d outside [0, %d)", device, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("cyl_sart_run_static: no address for the static scratch on device %d: %s", device,
                      hipGetErrorString(e));
            return nullptr;
        }
        scratch_dev[device] = p;
    }
    return scratch_dev[device];
}

extern "C" int cyl_sart_run_static(const cyl_geom *G, const cyl_sart_params *P, const void *proj, cyl_dtype pt,
                                   const void *pw, cyl_dtype pwt, const void *vw, cyl_dtype vwt, void *vol,
                                   cyl_dtype vt, void *hip_stream) {
    int rc;
    if ((rc = sart_check("cyl_sart_run_static", G, P, proj, pt, pw, pwt, vw, vwt, vol, vt))) return rc;
    const size_t need = cyl_sart_workspace_bytes(G, P);
    if (need > CYL_SART_STATIC_SCRATCH_BYTES) {
        set_error("cyl_sart_run_static: the geometry needs %zu bytes of scratch, above the static %zu", need,
                  (size_t)CYL_SART_STATIC_SCRATCH_BYTES);
        return CYL_EINVAL;
    }
    if (P->start_iter >= P->n_iter) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sart_run_static: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    void *ws = scratch_ptr(G->device);
    if (!ws) return CYL_EDEVICE;
    return sart_sweep(G, P, proj, pt, pw, pwt, vw, vwt, vol, vt, (float *)ws, (hipStream_t)hip_stream,
                      "cyl_sart_run_static");
}

// Residual images of one subset, then the view order as int32.
static size_t os_rho_bytes(const cyl_geom *G, int m) {
    return ((size_t)m * ((size_t)G->rows * G->cols + tile_count(G->dev)) * sizeof(float) + 255) & ~(size_t)255;
}

extern "C" size_t cyl_os_sart_workspace_bytes(const cyl_geom *G, int32_t subset) {
    if (!G || subset < 1) return 0;
    const int m = std::min(subset, G->n_views);
    return os_rho_bytes(G, m) + (((size_t)G->n_views * sizeof(int32_t) + 255) & ~(size_t)255);
}

extern "C" int cyl_os_sart_run(const cyl_geom *G, const cyl_sart_params *P, int32_t subset, const void *proj,
                               cyl_dtype pt, const void *pw, cyl_dtype pwt, const void *vw, cyl_dtype vwt,
                               void *vol, cyl_dtype vt, void *workspace, size_t ws_bytes, void *hip_stream) {
    int rc;
    if ((rc = sart_check("cyl_os_sart_run", G, P, proj, pt, pw, pwt, vw, vwt, vol, vt))) return rc;
    if (subset < 1) {
        set_error("cyl_os_sart_run: subset must be >= 1 (got %d)", subset);
        return CYL_EINVAL;
    }
    const int m = std::min(subset, G->n_views);
    if ((int64_t)m * G->rows * G->cols > (1LL << 28)) {
        set_error("cyl_os_sart_run: a subset of %d views of %d x %d pixels exceeds 2^28 rays", m, G->rows, G->cols);
        return CYL_EINVAL;
    }
    if (P->start_view % m != 0 && P->start_view != G->n_views) {
        set_error("cyl_os_sart_run: start_view %d is not at a subset boundary (subset %d)", P->start_view, m);
        return CYL_EINVAL;
    }
    const size_t need = cyl_os_sart_workspace_bytes(G, subset);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_os_sart_run: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    if (P->start_iter >= P->n_iter) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_os_sart_run: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    float *rho = (float *)workspace;
    int32_t *dlist = (int32_t *)((char *)workspace + os_rho_bytes(G, m));
    std::vector<int32_t> order(G->n_views);
    for (int i = 0; i < G->n_views; ++i) order[i] = P->view_order ? P->view_order[i] : i;
    store_i32(dlist, order.data(), G->n_views, st);
    const float lam = (float)P->lambda;
    for (int it = P->start_iter; it < P->n_iter; ++it) {
        const int kv0 = (it == P->start_iter) ? P->start_view : 0;
        for (int kk = kv0; kk < G->n_views; kk += m) {
            const int cnt = std::min(m, G->n_views - kk);
            launch_fp_views(G, vol, vt, const_cast<void *>(proj), pt, order.data() + kk, cnt, pw, pwt, rho, st);
            launch_bp(G, nullptr, CYL_F32, kk, kk + cnt, vol, vt, 0, true, rho, vw, vwt, lam, P->nonneg, st,
                      dlist);
        }
        if ((rc = launch_check("cyl_os_sart_run"))) return rc;
    }
    return CYL_OK;
}

extern "C" int cyl_sart_residual(const cyl_geom *G, int32_t view, const void *proj, cyl_dtype pt, const void *pw,
                                 cyl_dtype pwt, const void *vol, cyl_dtype vt, void *workspace, size_t ws_bytes,
                                 void *hip_stream) {
    if (!G || !proj || !vol) {
        set_error("cyl_sart_residual: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_sart_residual volume")) ||
        (rc = check_dtype(pt, "cyl_sart_residual projections")))
        return rc;
    if (pw && (rc = check_dtype(pwt, "cyl_sart_residual projection weights"))) return rc;
    if (view < 0 || view >= G->n_views) {
        set_error("cyl_sart_residual: view %d outside [0, %d)", view, G->n_views);
        return CYL_EINVAL;
    }
    const size_t need = cyl_sart_workspace_bytes(G, nullptr);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_sart_residual: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sart_residual: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_fp(G, vol, vt, const_cast<void *>(proj), pt, view, 1, true, pw, pwt, (float *)workspace,
              (hipStream_t)hip_stream);
    return launch_check("cyl_sart_residual");
}

extern "C" int cyl_sart_update(const cyl_geom *G, int32_t view, double lambda, int32_t nonneg, const void *vw,
                               cyl_dtype vwt, void *vol, cyl_dtype vt, const void *workspace, size_t ws_bytes,
                               void *hip_stream) {
    if (!G || !vol) {
        set_error("cyl_sart_update: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_sart_update volume"))) return rc;
    if (vw && (rc = check_dtype(vwt, "cyl_sart_update voxel weights"))) return rc;
    if (view < 0 || view >= G->n_views) {
        set_error("cyl_sart_update: view %d outside [0, %d)", view, G->n_views);
        return CYL_EINVAL;
    }
    if (!std::isfinite(lambda)) {
        set_error("cyl_sart_update: lambda must be finite");
        return CYL_EINVAL;
    }
    const size_t need = cyl_sart_workspace_bytes(G, nullptr);
    if (!workspace || ws_bytes < need) {
        set_error("cyl_sart_update: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return CYL_EINVAL;
    }
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_sart_update: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_bp(G, nullptr, CYL_F32, view, view + 1, vol, vt, 0, true, (const float *)workspace, vw, vwt,
              (float)lambda, nonneg, (hipStream_t)hip_stream);
    return launch_check("cyl_sart_update");
}

extern "C" int cyl_sart_batch_step(int32_t n, const cyl_sart_batch_item *items, cyl_dtype pt, cyl_dtype pwt,
                                   cyl_dtype vwt, cyl_dtype vt, void *hip_stream) {
    if (n < 0 || (n > 0 && !items)) {
        set_error("cyl_sart_batch_step: need n >= 0 and an items array");
        return CYL_EINVAL;
    }
    if (n == 0) return CYL_OK;
    int rc;
    if ((rc = check_dtype(vt, "cyl_sart_batch_step volume")) ||
        (rc = check_dtype(pt, "cyl_sart_batch_step projections")))
        return rc;
    bool any_pw = false, any_vw = false;
    for (int i = 0; i < n; ++i) {
        const cyl_sart_batch_item &it = items[i];
        if (!it.geom || !it.proj || !it.vol) {
            set_error("cyl_sart_batch_step: item %d has a NULL geometry, projection or volume", i);
            return CYL_EINVAL;
        }
        if (it.geom->device != items[0].geom->device) {
            set_error("cyl_sart_batch_step: item %d is on device %d, item 0 on %d", i, it.geom->device,
                      items[0].geom->device);
            return CYL_EINVAL;
        }
        if (it.view < 0 || it.view >= it.geom->n_views) {
            set_error("cyl_sart_batch_step: item %d view %d outside [0, %d)", i, it.view, it.geom->n_views);
            return CYL_EINVAL;
        }
        const size_t need = cyl_sart_workspace_bytes(it.geom, nullptr);
        if (!it.workspace || it.workspace_bytes < need) {
            set_error("cyl_sart_batch_step: item %d workspace of %zu bytes is smaller than the %zu needed", i,
                      it.workspace_bytes, need);
            return CYL_EINVAL;
        }
        if (!std::isfinite(it.lambda)) {
            set_error("cyl_sart_batch_step: item %d lambda must be finite", i);
            return CYL_EINVAL;
        }
        any_pw |= it.proj_weights != nullptr;
        any_vw |= it.vox_weights != nullptr;
    }
    if (any_pw && (rc = check_dtype(pwt, "cyl_sart_batch_step projection weights"))) return rc;
    if (any_vw && (rc = check_dtype(vwt, "cyl_sart_batch_step voxel weights"))) return rc;
    DeviceGuard dg(items[0].geom->device);
    if (!dg.ok) {
        set_error("cyl_sart_batch_step: cannot select device %d", items[0].geom->device);
        return CYL_EDEVICE;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    const cyl_geom *geoms[kMaxBatch];
    for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
        FpLaunch L;
        L.n = std::min(kMaxBatch, n - i0);
        for (int i = 0; i < L.n; ++i) {
            const cyl_sart_batch_item &it = items[i0 + i];
            L.item[i] = fp_item(it.geom, it.vol, const_cast<void *>(it.proj), it.view, fp_split(it.geom->dev, 1),
                                it.proj_weights, pwt, (float *)it.workspace,
                                (float *)it.workspace + (size_t)it.geom->rows * it.geom->cols);
            geoms[i] = it.geom;
        }
        launch_fp_batch(L, geoms, vt, pt, true, st);
    }
    for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
        BpLaunch L;
        L.n = std::min(kMaxBatch, n - i0);
        for (int i = 0; i < L.n; ++i) {
            const cyl_sart_batch_item &it = items[i0 + i];
            L.item[i] = bp_item(it.geom, it.workspace, it.view, it.view + 1, it.vol, 0, it.vox_weights, vwt,
                                (float)it.lambda, it.nonneg);
            geoms[i] = it.geom;
        }
        launch_bp_batch(L, geoms, vt, CYL_F32, true, st);
    }
    return launch_check("cyl_sart_batch_step");
}

extern "C" int cyl_fp_diff(const cyl_geom *G, const void *vol, cyl_dtype vt, const void *base, cyl_dtype bt,
                           void *out, cyl_dtype ot, int32_t view_begin, int32_t view_end, void *hip_stream) {
    if (!G || !vol || !base || !out) {
        set_error("cyl_fp_diff: NULL argument");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(vt, "cyl_fp_diff volume")) || (rc = check_dtype(bt, "cyl_fp_diff base projections")) ||
        (rc = check_dtype(ot, "cyl_fp_diff output")) || (rc = check_range(G, view_begin, view_end, "cyl_fp_diff")))
        return rc;
    if (view_end == view_begin) return CYL_OK;
    DeviceGuard dg(G->device);
    if (!dg.ok) {
        set_error("cyl_fp_diff: cannot select device %d", G->device);
        return CYL_EDEVICE;
    }
    launch_fp(G, vol, vt, out, ot, view_begin, view_end - view_begin, false, base, bt, nullptr,
              (hipStream_t)hip_stream);
    return launch_check("cyl_fp_diff");
}

extern "C" int cyl_add(int64_t n, const void *a, cyl_dtype at, const void *b, cyl_dtype bt, void *out,
                       cyl_dtype ot, int32_t device, void *hip_stream) {
    if (n < 0 || (n > 0 && (!a || !b || !out))) {
        set_error("cyl_add: need n >= 0 and non-NULL arrays");
        return CYL_EINVAL;
    }
    int rc;
    if ((rc = check_dtype(at, "cyl_add a")) || (rc = check_dtype(bt, "cyl_add b")) ||
        (rc = check_dtype(ot, "cyl_add out")))
        return rc;
    if (n == 0) return CYL_OK;
    DeviceGuard dg(device);
    if (!dg.ok) {
        set_error("cyl_add: cannot select device %d", device);
        return CYL_EDEVICE;
    }
    const size_t blocks = std::min<size_t>(((size_t)n + 255) / 256, 8192);
    hipStream_t st = (hipStream_t)hip_stream;
    switch (ot) {
        case CYL_F32: hipLaunchKernelGGL(add_kernel<CYL_F32>, dim3(blocks), dim3(256), 0, st, (size_t)n, a, at, b, bt, out); break;
        case CYL_F16: hipLaunchKernelGGL(add_kernel<CYL_F16>, dim3(blocks), dim3(256), 0, st, (size_t)n, a, at, b, bt, out); break;
        default: hipLaunchKernelGGL(add_kernel<CYL_BF16>, dim3(blocks), dim3(256), 0, st, (size_t)n, a, at, b, bt, out); break;
    }
    return launch_check("cyl_add");
}
