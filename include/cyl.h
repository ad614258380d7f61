/*
 * cyl.h — C ABI of libcyl: cone-beam forward projection, its exact transpose
 * and weighted SART on an object-fixed cylindrical voxel grid, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Paper: "Fast tomographic inspection of cylindrical objects" (arXiv 2005.11976).
 *   Sec. 2, Eq. 1    object pose  X' = R X + T  (stage frame X -> object frame X')
 *   Sec. 2, Eq. 2    cylindrical cells:  r = sqrt(x'^2 + y'^2), theta = atan2(y', x'),
 *                    h = z'  (the printed arctan(y'/x') is read as the two-argument
 *                    arctangent taken modulo 2 pi)
 *   Sec. 2.2, Eq. 6  p_j = sum_l t_jl mu_l, t_jl = length of ray j inside cell l
 *   Sec. 2.2, Eq. 7  SART update per projection with relaxation lambda, row sums
 *                    sum_l t_jl and column sums sum_j t_jm
 *   Sec. 2.2, last paragraph: voxel weight map (weighted back-projection);
 *   Sec. 1 and 3.3:  prior (initial) volume.
 *
 * Conventions shared by every entry point
 *   - lengths in mm, angles in radians, attenuation in 1/mm;
 *   - grid: r_i = r_min + i (r_max - r_min)/n_r, h_m = h_min + m (h_max - h_min)/n_h,
 *     theta_b = theta0 + 2 pi b / n_theta; every cell is half-open [lower, upper);
 *   - volumes are C-ordered [n_h][n_theta][n_r] (r fastest);
 *   - projections are C-ordered [n_views][det_rows][det_cols];
 *   - ray j = (view k, row v, col u) runs from the source S_k to the pixel centre
 *     D_k + (u - (det_cols-1)/2) U_k + (v - (det_rows-1)/2) V_k (one ray per pixel);
 *   - every array argument except cyl_traj.views and cyl_sart_params.view_order is
 *     a DEVICE pointer owned by the caller (e.g. the storage of a contiguous torch
 *     tensor on the geometry's device); the library never frees caller memory;
 *   - calls validate their arguments, enqueue work on `hip_stream` (a hipStream_t,
 *     NULL = the default stream) and return before the work completes.  A failed
 *     validation returns CYL_EINVAL, enqueues nothing and sets cyl_last_error().
 *     A launch failure returns CYL_EDEVICE.  Faults inside kernels surface at the
 *     caller's next synchronisation of the stream;
 *   - a cyl_geom is immutable after creation, so several streams and threads may
 *     share it; calls that write the same buffer must be ordered by the caller.
 */
#ifndef CYL_H
#define CYL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cyl_geom cyl_geom; /* opaque */

/* Storage types of volumes, projections and weights.  Arithmetic is always
 * FP32 (FP64 for the per-ray set-up and the row sums); FP16/BF16 values are
 * widened on load and rounded to nearest-even on store. */
typedef enum { CYL_F32 = 0, CYL_F16 = 1, CYL_BF16 = 2 } cyl_dtype;

enum {
    CYL_OK = 0,
    CYL_EINVAL = -1,      /* invalid argument; nothing enqueued */
    CYL_ENOMEM = -2,      /* device allocation failed */
    CYL_EDEVICE = -3,     /* HIP runtime or launch error */
    CYL_EUNSUPPORTED = -4 /* valid but not supported by this build */
};

/* Cylindrical grid in the object frame (Sec. 2, Eq. 2).
 * Requires n_h, n_theta, n_r >= 1, 0 <= r_min < r_max, h_min < h_max, at most
 * 2^30 - 1 cells (volume byte offsets are 32-bit) and n_theta * n_r < 2^24
 * (cell indices are formed with 24-bit products). */
typedef struct {
    int32_t n_h, n_theta, n_r;
    double r_min, r_max;
    double h_min, h_max;
    double theta0; /* lower edge of sector 0 */
} cyl_grid;

/* Source/detector trajectory (Sec. 2.1 and Table 1: circular or any other
 * trajectory; Sec. 1 mentions conveyor belts).  One 12-vector per view in the
 * STAGE frame: source[3], detector centre[3], pixel step along a row (u)[3],
 * pixel step along a column (v)[3].  `views` is a HOST pointer, read during
 * cyl_geom_create only.  Requires n_views, det_rows, det_cols >= 1 and a
 * non-degenerate detector (u and v steps not parallel, source off the
 * detector plane). */
typedef struct {
    int32_t n_views, det_rows, det_cols;
    const double *views;
} cyl_traj;

/* Rigid pose of the object (Sec. 2, Eq. 1): X' = R X + T, R row-major.  R must
 * be a rotation (orthonormal to 1e-9, det +1). */
typedef struct {
    double R[9];
    double T[3];
} cyl_pose;

/* Builds the immutable geometry on HIP device `device`: validates the inputs,
 * maps every view into the object frame in FP64 (Eq. 1 applied once per view,
 * the paper's precomputed alignment, Sec. 2.2) and uploads the grid tables.
 * Fails with CYL_EINVAL if any source point lies inside the grid support
 * (r < r_max and h_min <= h < h_max in the object frame).  Device memory owned
 * by the geometry: a few hundred bytes per view plus the grid tables; freed by
 * cyl_geom_destroy.  *out is set only on success. */
int cyl_geom_create(const cyl_grid *grid, const cyl_traj *traj, const cyl_pose *pose,
                    int device, cyl_geom **out);

/* Frees the geometry (NULL is ignored).  The caller must make sure no enqueued
 * work still uses it. */
void cyl_geom_destroy(cyl_geom *geom);

/* Forward projection (Eq. 6): proj[k][v][u] = sum_l t_jl vol_l for the views
 * k in [view_begin, view_end).  `vol` is the full volume; `proj` is the full
 * [n_views][rows][cols] array of which only those views are written.  t_jl is
 * the exact length of the source -> pixel-centre segment inside cell l,
 * accumulated in FP32 along the ray.  An empty range is a no-op. */
int cyl_fp(const cyl_geom *geom, const void *vol, cyl_dtype vol_type, void *proj,
           cyl_dtype proj_type, int32_t view_begin, int32_t view_end, void *hip_stream);

/* Back-projection, the exact transpose of cyl_fp:
 * vol_l = (accumulate ? vol_l : 0) + sum_{k in range} sum_j t_jl proj_j.
 * No normalisation.  `proj` is the full [n_views][rows][cols] array of which
 * only the views in range are read.  Deterministic: no global atomics; every
 * voxel is written once by the wave that owns it. */
int cyl_bp(const cyl_geom *geom, const void *proj, cyl_dtype proj_type, void *vol,
           cyl_dtype vol_type, int32_t view_begin, int32_t view_end, int32_t accumulate,
           void *hip_stream);

/* Row sums L_j = sum_l t_jl (Eq. 7 denominator) in closed form: the length of
 * the ray inside the support r_min <= r < r_max, h_min <= h < h_max, computed
 * in FP64 per ray and stored as FP32 into the full [n_views][rows][cols]
 * array `out` for the views in range. */
int cyl_row_sums(const cyl_geom *geom, float *out, int32_t view_begin, int32_t view_end,
                 void *hip_stream);

/* SART parameters (Eq. 7).  One update step per projection (the ordered subset
 * is one view); one iteration sweeps all views in `view_order` (HOST pointer to
 * n_views indices, each in [0, n_views); NULL = 0 .. n_views-1).  Resume: start
 * at iteration start_iter, position start_view of the order (0, 0 = fresh).
 * nonneg != 0 clamps mu at 0 after every update. */
typedef struct {
    int32_t n_iter;
    double lambda;
    int32_t nonneg;
    const int32_t *view_order;
    int32_t start_iter, start_view;
} cyl_sart_params;

/* Device workspace bytes cyl_sart_run needs for this geometry: the FP32
 * residual image of one view ([rows][cols]), then the largest |rho| of each
 * aligned 8x8 pixel tile of that image ([ceil(rows/8)][ceil(cols/8)] FP32,
 * which bounds the update's fixed-point sums), rounded up to 256 bytes. */
size_t cyl_sart_workspace_bytes(const cyl_geom *geom, const cyl_sart_params *params);

/* Weighted SART from a prior (Eq. 7; weight map Sec. 2.2; prior Sec. 1, 3.3).
 * For each iteration and each view k in order:
 *   q_j   = sum_l t_jl mu_l                          (FP32 along the ray)
 *   rho_j = wp_j (p_j - q_j) / L_j   if L_j > 0 else 0   (L_j: closed-form row sum)
 *   c_m   = sum_{j in k} t_jm rho_j,  n_m = sum_{j in k} t_jm
 *   mu_m += lambda * wv_m * c_m / n_m   if n_m > 0    (rounded into vol_type)
 * proj: measured line integrals p (Eq. 6), [n_views][rows][cols].
 * proj_weights: per-pixel weights wp, same layout, or NULL (all 1).
 * vox_weights: per-voxel weights wv (volume layout), or NULL (all 1).
 * vol: in = prior mu(0), out = result, updated in place.
 * workspace: device buffer of at least cyl_sart_workspace_bytes() bytes, owned
 * by the caller, not used by anything else until the work completes. */
int cyl_sart_run(const cyl_geom *geom, const cyl_sart_params *params, const void *proj,
                 cyl_dtype proj_type, const void *proj_weights, cyl_dtype proj_weights_type,
                 const void *vox_weights, cyl_dtype vox_weights_type, void *vol,
                 cyl_dtype vol_type, void *workspace, size_t workspace_bytes,
                 void *hip_stream);

/* cyl_sart_run for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  Computes
 * exactly what cyl_sart_run computes (the same kernels, bit for bit), with the
 * library's own static device scratch (CYL_SART_STATIC_SCRATCH_BYTES per GPU,
 * held until the process ends) in place of the caller's workspace.  The caller
 * still passes proj, the weights and vol; arguments as for cyl_sart_run.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); it fails with CYL_EINVAL, enqueuing nothing, when the geometry's
 * workspace (cyl_sart_workspace_bytes) exceeds the scratch, which holds the
 * workspace of a 1024 x 1024 detector (1024 x 768 fits).  Every call on one GPU shares
 * that GPU's scratch, so calls that overlap on one GPU (other streams or
 * threads) race: the caller must order them.  The scratch keeps the last
 * call's contents; every residual and tile maximum a call reads it has
 * written first in the same call. */
#define CYL_SART_STATIC_SCRATCH_BYTES ((size_t)4259840) /* (2^20 + 2^14) FP32 words */
int cyl_sart_run_static(const cyl_geom *geom, const cyl_sart_params *params, const void *proj,
                        cyl_dtype proj_type, const void *proj_weights, cyl_dtype proj_weights_type,
                        const void *vox_weights, cyl_dtype vox_weights_type, void *vol,
                        cyl_dtype vol_type, void *hip_stream);

/* Ordered-subset SART (Eq. 7 with an ordered subset of several projections;
 * subset = n_views is SIRT).  Each iteration splits the view order into
 * consecutive groups of `subset` positions (the last group may be shorter);
 * per group, all its views are projected from the same mu, then
 *   rho_j = wp_j (p_j - q_j) / L_j                  for every ray of the group
 *   c_m   = sum_{j in group} t_jm rho_j,  n_m = sum_{j in group} t_jm
 *   mu_m += lambda * wv_m * c_m / n_m   if n_m > 0  (rounded into vol_type)
 * subset = 1 computes exactly what cyl_sart_run computes, bit for bit.
 * Arguments as for cyl_sart_run, plus:
 *   subset     views per update, >= 1 (values above n_views act as n_views);
 *              subset x rows x cols must not exceed 2^28 rays
 *   workspace  device buffer of at least cyl_os_sart_workspace_bytes(geom,
 *              subset) bytes (one FP32 residual image per view of a group,
 *              then their 8x8 tile maxima, then the view order), owned by
 *              the caller, not used by anything
 *              else until the work completes
 * A resume point (start_view) must fall on a group boundary.  Errors:
 * CYL_EINVAL for bad arguments (nothing is launched), CYL_EDEVICE for launch
 * failures. */
size_t cyl_os_sart_workspace_bytes(const cyl_geom *geom, int32_t subset);
int cyl_os_sart_run(const cyl_geom *geom, const cyl_sart_params *params, int32_t subset, const void *proj,
                    cyl_dtype proj_type, const void *proj_weights, cyl_dtype proj_weights_type,
                    const void *vox_weights, cyl_dtype vox_weights_type, void *vol, cyl_dtype vol_type,
                    void *workspace, size_t workspace_bytes, void *hip_stream);

/* The two kernels of one SART sub-iteration (Eq. 7, one view), for callers
 * that schedule views themselves (a serving loop interleaving scans, or a
 * profiler timing each kernel).  Running, for k in order,
 * cyl_sart_residual(k) then cyl_sart_update(k) on one stream is exactly
 * cyl_sart_run.
 * cyl_sart_residual: rho_j = wp_j (p_j - sum_l t_jl mu_l) / L_j for the rays of
 *   view `view`, written as FP32 into `workspace` ([rows][cols], then the
 *   largest |rho| of each aligned 8x8 tile).
 * cyl_sart_update: c_m = sum_j t_jm rho_j, n_m = sum_j t_jm over that view's
 *   rays; mu_m += lambda wv_m c_m / n_m where n_m > 0 (clamped at 0 if nonneg).
 * Arguments as for cyl_sart_run; workspace of cyl_sart_workspace_bytes(). */
int cyl_sart_residual(const cyl_geom *geom, int32_t view, const void *proj, cyl_dtype proj_type,
                      const void *proj_weights, cyl_dtype proj_weights_type, const void *vol,
                      cyl_dtype vol_type, void *workspace, size_t workspace_bytes, void *hip_stream);
int cyl_sart_update(const cyl_geom *geom, int32_t view, double lambda, int32_t nonneg,
                    const void *vox_weights, cyl_dtype vox_weights_type, void *vol, cyl_dtype vol_type,
                    const void *workspace, size_t workspace_bytes, void *hip_stream);

/* out[k] = base[k] - A_k vol for views k in [view_begin, view_end): given
 * projections minus the forward projection of a volume (Eq. 6), formed in FP32
 * and rounded once into out_type.  With vol = the prior it gives the data of
 * SART run on the difference from the prior (Sec. 2.2 starts from a prior):
 * SART from mu(0) on p equals mu(0) + SART from 0 on p - A mu(0), and the
 * difference and its projections are small, so FP16/BF16 storage holds them
 * with little error.  Layouts as cyl_fp; base and out may be the same buffer.
 * Errors as cyl_fp. */
int cyl_fp_diff(const cyl_geom *geom, const void *vol, cyl_dtype vol_type, const void *base,
                cyl_dtype base_type, void *out, cyl_dtype out_type, int32_t view_begin,
                int32_t view_end, void *hip_stream);

/* out = a + b over n values of device memory on HIP device `device`
 * (storage types a_type, b_type, out_type; FP32 arithmetic, rounded to
 * nearest-even on store); out may alias a or b.  Used to form prior + difference
 * volumes.  CYL_EINVAL for n < 0 or a NULL array. */
int cyl_add(int64_t n, const void *a, cyl_dtype a_type, const void *b, cyl_dtype b_type, void *out,
            cyl_dtype out_type, int32_t device, void *hip_stream);

/* One SART sub-iteration (Eq. 7 with the ordered subset = one projection,
 * Sec. 2.2) for each of n independent scans, in two launches: the forward
 * projections with residuals of all items, then their back-projections with
 * updates.  Serving uses it to run scans that arrive over time side by side
 * (different grids, poses and detectors); item i computes exactly what
 * cyl_sart_residual(view) + cyl_sart_update(view) compute for it alone, bit for
 * bit, whatever else is in the batch.
 *   items[i].geom       geometry of scan i; all geometries on one device
 *   items[i].view       view of this sub-iteration, in [0, n_views)
 *   items[i].proj       measured projections of scan i, all views, proj_type
 *   items[i].proj_weights / vox_weights   per-pixel / per-voxel weights or NULL
 *   items[i].vol        volume of scan i, updated in place, vol_type
 *   items[i].workspace  >= cyl_sart_workspace_bytes(geom) bytes of device memory
 * Storage types are common to the batch.  Volumes and workspaces of different
 * items must not overlap (they are written concurrently).  n = 0 is a no-op;
 * any n >= 1 is accepted (launched in groups of 16 items).  Errors: CYL_EINVAL
 * for a NULL items array or field, a view out of range, a small workspace,
 * mixed devices or a non-finite lambda (nothing enqueued). */
typedef struct {
    const cyl_geom *geom;
    int32_t view;
    const void *proj;
    const void *proj_weights;
    const void *vox_weights;
    void *vol;
    void *workspace;
    size_t workspace_bytes;
    double lambda;
    int32_t nonneg;
} cyl_sart_batch_item;

int cyl_sart_batch_step(int32_t n, const cyl_sart_batch_item *items, cyl_dtype proj_type,
                        cyl_dtype proj_weights_type, cyl_dtype vox_weights_type, cyl_dtype vol_type,
                        void *hip_stream);

/* ---- pose estimation from projections (Sec. 2.1) ---------------------- */

/* Corner pixels of the segmented object in each projection (axis tracking):
 * pixels whose value exceeds `threshold` (rounded to FP32), dilated by a square
 * of half-width `dilate`; with u the column and v the row index, the corners
 * are top-left = min u+v, top-right = max u-v (ties: smallest v), bottom-left =
 * min u-v, bottom-right = max u+v (ties: largest v).  The pairwise centres of
 * the two top and the two bottom corners are two points of the projected
 * symmetry axis.
 *   proj     device, [n_views][rows][cols] of proj_type
 *   corners  device int32, [n_views][9]: TL.u TL.v TR.u TR.v BL.u BL.v BR.u BR.v
 *            and the number of pixels above the threshold; the corners are -1
 *            for a view with none.
 * Exact integer results (independent of the reduction order).  CYL_EINVAL for
 * bad sizes or NULL buffers; asynchronous on hip_stream of device `device`. */
int cyl_axis_corners(int32_t n_views, int32_t rows, int32_t cols, const void *proj, cyl_dtype proj_type,
                     double threshold, int32_t dilate, int32_t *corners, int32_t device, void *hip_stream);

/* Point tracking, Eq. 3-4: the stage-frame point X minimising
 * sum_k |uv_k - V_k(X)|^2 over the views k with valid[k] != 0 (valid may be
 * NULL = all), V_k the cone-beam projection of view k to detector coordinates
 * (u = column, v = row, pixel centres at integers).  Levenberg-Marquardt with
 * analytic derivatives from the least-squares intersection of the views'
 * rays.  Host call on host arrays: uv [n_views][2]; writes xyz[3] and, if rms
 * is not NULL, the root-mean-square residual in pixels.  CYL_EINVAL for fewer
 * than two valid views, non-finite points or a degenerate detector. */
int cyl_track_point(const cyl_traj *traj, const double *uv, const uint8_t *valid, double *xyz, double *rms);

/* Pose (Eq. 1, X' = R X + T with R = Rz(alpha) Rx(beta) Rz(gamma)) from two
 * stage-frame points of the object's symmetry axis at object heights
 * h_top > h_bottom, and the internal rotation angle alpha about that axis:
 * beta and gamma follow from the axis direction R^T z, and the object origin
 * (the axis point at height 0) from the points' midpoint.  Host call.
 * CYL_EINVAL for coincident points, h_top <= h_bottom or non-finite values. */
int cyl_pose_from_axis(const double *top, const double *bottom, double h_top, double h_bottom, double alpha,
                       cyl_pose *out);

/* Grey values beside the projected axis (Sec. 2.1, azimuthal phase): for each
 * view k, over rows [row_lo[k], row_hi[k]] (clipped to the detector),
 * sums[2k] = sum of the pixels left of detector position centre[k] and
 * sums[2k+1] = sum right of it; pixel u spans [u - 1/2, u + 1/2] and is split
 * at the centre in proportion.  All arrays are device memory: proj
 * [n_views][rows][cols] of proj_type, centre float64 [n_views], row_lo/row_hi
 * int32 [n_views], sums float64 [n_views][2].  FP64 accumulation in a fixed
 * order (reproducible).  CYL_EINVAL for bad sizes or NULL buffers. */
int cyl_side_sums(int32_t n_views, int32_t rows, int32_t cols, const void *proj, cyl_dtype proj_type,
                  const double *centre, const int32_t *row_lo, const int32_t *row_hi, double *sums,
                  int32_t device, void *hip_stream);

/* Internal rotation angle (Sec. 2.1, Eq. 5) from a measured grey-value signal s
 * and a reference signal s_ref, both sampled at the n equally spaced view
 * angles of a full circular trajectory, the reference projected with the same
 * axis pose and no internal rotation: the angle a in [0, 2 pi) maximising the
 * circular cross-correlation of s(phi) and s_ref(phi + a) (a view-angle shift
 * is a rotation of the object about the rotation axis; the reference carries
 * the tilt correction of Eq. 5).  Trigonometric interpolation through the
 * discrete Fourier coefficients m = 1 .. (n-1)/2, best of a 0.1-degree grid
 * refined by Newton steps.  Host call.  CYL_EINVAL for n < 3, NULL arrays or
 * non-finite values. */
int cyl_azimuth_phase(int32_t n, const double *s, const double *s_ref, double *alpha);

/* Sec. 2.1, Eq. 5: the object's last Euler angle from the perceived phase
 * phi_p of the grey-value signal, the geometric angle phi_g of the scanner's
 * optical axis and the first two Euler angles a1, a2 of Eq. 1 (the paper's
 * alpha and beta): gamma = phi_p - phi_g - arctan(tan(a1) / cos(a2)), the
 * arctangent taken as atan2(sin a1, cos a1 cos a2) so that it stays continuous
 * through a1 = +-pi/2; gamma is wrapped to [0, 2 pi).  Host call.  CYL_EINVAL
 * for a NULL output, non-finite arguments or cos(a2) = 0. */
int cyl_gamma_from_phase(double phi_p, double phi_g, double a1, double a2, double *gamma);

/* The two points of the projected symmetry axis per view from the output of
 * cyl_axis_corners (Sec. 2.1): top = centre of the top-left and top-right
 * corners, bottom = centre of the bottom-left and bottom-right ones, as
 * (u, v) pixel coordinates; valid[k] = 1 where view k has pixels above the
 * threshold, else 0 (and its points are -1).  Host call on host arrays:
 * corners [n_views][9] (int32, as written by cyl_axis_corners), top and bottom
 * [n_views][2], valid [n_views].  CYL_EINVAL for n_views < 1 or NULL arrays. */
int cyl_axis_points(int32_t n_views, const int32_t *corners, double *top, double *bottom, uint8_t *valid);

/* The paper's own projector pair (Sec. 2.2), for comparison with the exact
 * pair above.  Forward projection, pixel driven: each ray (source -> pixel
 * centre) is sampled at distances (k + 1/2) step from the source; each sample
 * inside the support goes through the cylindrical transform (Eq. 2) and adds
 * step * mu, with mu of the cell holding it (interp = 0: t_jl = step x samples
 * in cell l) or interpolated trilinearly between cell centres (interp = 1;
 * theta periodic, r and h clamped to the outermost centres).  Row sums are
 * step x (samples in the support).  FP32.  step in mm, > 0, with at most
 * 2^30 samples across the support.  Views [view_begin, view_end) of proj
 * ([n_views][rows][cols]) are overwritten. */
int cyl_fp_sampled(const cyl_geom *geom, const void *vol, cyl_dtype vol_type, void *proj, cyl_dtype proj_type,
                   int32_t view_begin, int32_t view_end, double step, int32_t interp, void *hip_stream);

/* Voxel-driven back-projection (Sec. 2.2): for each cell, the bilinear reading
 * of each view's image at the projection of the cell centre (pixels off the
 * detector read nothing), summed over views [view_begin, view_end) of proj
 * ([n_views][rows][cols]); vol = (accumulate ? vol : 0) + that sum.  Not the
 * transpose of cyl_fp_sampled.  FP32. */
int cyl_bp_voxel(const cyl_geom *geom, const void *proj, cyl_dtype proj_type, void *vol, cyl_dtype vol_type,
                 int32_t view_begin, int32_t view_end, int32_t accumulate, void *hip_stream);

/* SART (Eq. 7, one projection per update) with the paper's pair: per view k,
 * rho = wp (p - q) / L from cyl_fp_sampled's q and row sums L, then
 * mu_m += lambda wv_m c_m / n_m with c the voxel-driven back-projection of rho
 * and n the bilinear weights that fell on the detector (where n > 0).
 * Parameters, buffers and workspace (cyl_sart_workspace_bytes) as for
 * cyl_sart_run, plus step and interp as for cyl_fp_sampled. */
int cyl_sart_run_sampled(const cyl_geom *geom, const cyl_sart_params *params, double step, int32_t interp,
                         const void *proj, cyl_dtype proj_type, const void *proj_weights,
                         cyl_dtype proj_weights_type, const void *vox_weights, cyl_dtype vox_weights_type, void *vol,
                         cyl_dtype vol_type, void *workspace, size_t workspace_bytes, void *hip_stream);

/* Precomputed system matrix for scans whose views are view 0 rotated about the
 * object axis by whole sectors (an unposed circular scan with a view step that
 * is a multiple of 2 pi / n_theta): the reuse of the system matrix that the
 * posed method gives up (Sec. 2).  cyl_sym_create checks the views on the host
 * (each must match view 0 rotated by an integer number of sectors within
 * 1e-9 of its size; CYL_EINVAL otherwise), then records view 0's exact rows
 * t_jl with the traversal and builds its columns (device memory: 10 bytes per
 * row entry, 8 per column entry, 8 per cell and per ray; it synchronises
 * `hip_stream`).  The geometry must outlive the matrix.  Entries per view must
 * stay below 2^31; n_theta <= 65535.
 * cyl_sym_fp: q for views [view_begin, view_end) from the stored rows with the
 *   view's theta shift (as cyl_fp computes, to rounding).
 * cyl_sym_sart_run: weighted SART as cyl_sart_run computes it (to rounding),
 *   from the stored rows and columns; same parameters, buffers and
 *   workspace (cyl_sart_workspace_bytes of the geometry).  Deterministic. */
typedef struct cyl_sym cyl_sym;
int cyl_sym_create(const cyl_geom *geom, cyl_sym **out, void *hip_stream);
void cyl_sym_destroy(cyl_sym *sym);
int64_t cyl_sym_nnz(const cyl_sym *sym);
int cyl_sym_fp(const cyl_sym *sym, const void *vol, cyl_dtype vol_type, void *proj, cyl_dtype proj_type,
               int32_t view_begin, int32_t view_end, void *hip_stream);
int cyl_sym_sart_run(const cyl_sym *sym, const cyl_sart_params *params, const void *proj, cyl_dtype proj_type,
                     const void *proj_weights, cyl_dtype proj_weights_type, const void *vox_weights,
                     cyl_dtype vox_weights_type, void *vol, cyl_dtype vol_type, void *workspace,
                     size_t workspace_bytes, void *hip_stream);

/* Directional MTF of a volume (Sec. 2.3, Eq. 8) on its central h-slice: the
 * middle slice, or the mean of the two middle slices when n_h is even, in
 * FP64.  Each output is the modulation m = (max - min) / (max + min) (0 when
 * max + min = 0) of a set of cells of that slice:
 *   window = 0: out[r] over ring r (all theta), r in [0, n_r): the azimuthal
 *               MTF at each radius;
 *   window = w: out[k] over the rings [k w, (k + 1) w), k in [0, n_r / w):
 *               the radial MTF in windows of one phantom period.
 * vol: device (n_h, n_theta, n_r) of vol_type; out: device float64 array of
 * n_r (window 0) or n_r / window entries.  Exact and order-independent.
 * CYL_EINVAL for bad sizes, window outside [0, n_r] or NULL buffers. */
int cyl_mtf(int32_t n_h, int32_t n_theta, int32_t n_r, const void *vol, cyl_dtype vol_type, int32_t window,
            double *out, int32_t device, void *hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char *cyl_last_error(void);

/* Library version string. */
const char *cyl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CYL_H */
