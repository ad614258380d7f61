"""Thin Python binding of libcyl (argument marshalling only).

Every step of the path runs in the HIP kernels of libcyl.so; this module only
turns torch tensors and scan descriptions into the C-ABI calls declared in
include/cyl.h.  It raises if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcyl.so")

CYL_F32, CYL_F16, CYL_BF16 = 0, 1, 2
SART_STATIC_SCRATCH_BYTES = 4259840  # CYL_SART_STATIC_SCRATCH_BYTES of include/cyl.h
CYL_OK, CYL_EINVAL, CYL_ENOMEM, CYL_EDEVICE, CYL_EUNSUPPORTED = 0, -1, -2, -3, -4

EXPORTS = ["cyl_geom_create", "cyl_geom_destroy", "cyl_fp", "cyl_bp", "cyl_row_sums",
           "cyl_sart_workspace_bytes", "cyl_sart_run", "cyl_sart_run_static", "cyl_os_sart_workspace_bytes", "cyl_os_sart_run",
           "cyl_sart_residual", "cyl_sart_update",
           "cyl_sart_batch_step", "cyl_fp_diff", "cyl_add", "cyl_axis_corners", "cyl_track_point",
           "cyl_pose_from_axis", "cyl_side_sums", "cyl_azimuth_phase", "cyl_gamma_from_phase", "cyl_axis_points", "cyl_mtf", "cyl_fp_sampled", "cyl_bp_voxel", "cyl_sart_run_sampled", "cyl_sym_create", "cyl_sym_destroy", "cyl_sym_nnz",
           "cyl_sym_fp", "cyl_sym_sart_run", "cyl_last_error", "cyl_version"]


class CylError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libcyl error %d: %s" % (code, msg))
        self.code = code


class cyl_grid(C.Structure):
    _fields_ = [("n_h", C.c_int32), ("n_theta", C.c_int32), ("n_r", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("h_min", C.c_double),
                ("h_max", C.c_double), ("theta0", C.c_double)]


class cyl_traj(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("det_rows", C.c_int32), ("det_cols", C.c_int32),
                ("views", C.POINTER(C.c_double))]


class cyl_pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("T", C.c_double * 3)]


class cyl_sart_params(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("lam", C.c_double), ("nonneg", C.c_int32),
                ("view_order", C.POINTER(C.c_int32)), ("start_iter", C.c_int32),
                ("start_view", C.c_int32)]


class cyl_sart_batch_item(C.Structure):
    _fields_ = [("geom", C.c_void_p), ("view", C.c_int32), ("proj", C.c_void_p),
                ("proj_weights", C.c_void_p), ("vox_weights", C.c_void_p), ("vol", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("lam", C.c_double),
                ("nonneg", C.c_int32)]


_lib = None


def declare(lib):
    """Attach argument/return types of the C ABI to a loaded library."""
    vp, i32, P = C.c_void_p, C.c_int32, C.POINTER
    lib.cyl_geom_create.argtypes = [P(cyl_grid), P(cyl_traj), P(cyl_pose), C.c_int, P(vp)]
    lib.cyl_geom_create.restype = C.c_int
    lib.cyl_geom_destroy.argtypes = [vp]
    lib.cyl_geom_destroy.restype = None
    lib.cyl_fp.argtypes = [vp, vp, C.c_int, vp, C.c_int, i32, i32, vp]
    lib.cyl_fp.restype = C.c_int
    lib.cyl_bp.argtypes = [vp, vp, C.c_int, vp, C.c_int, i32, i32, i32, vp]
    lib.cyl_bp.restype = C.c_int
    lib.cyl_row_sums.argtypes = [vp, vp, i32, i32, vp]
    lib.cyl_row_sums.restype = C.c_int
    lib.cyl_sart_workspace_bytes.argtypes = [vp, P(cyl_sart_params)]
    lib.cyl_sart_workspace_bytes.restype = C.c_size_t
    lib.cyl_sart_run.argtypes = [vp, P(cyl_sart_params), vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                 vp, C.c_int, vp, C.c_size_t, vp]
    lib.cyl_sart_run.restype = C.c_int
    lib.cyl_sart_run_static.argtypes = [vp, P(cyl_sart_params), vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                        vp, C.c_int, vp]
    lib.cyl_sart_run_static.restype = C.c_int
    lib.cyl_os_sart_workspace_bytes.argtypes = [vp, i32]
    lib.cyl_os_sart_workspace_bytes.restype = C.c_size_t
    lib.cyl_os_sart_run.argtypes = [vp, P(cyl_sart_params), i32, vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                    vp, C.c_int, vp, C.c_size_t, vp]
    lib.cyl_os_sart_run.restype = C.c_int
    lib.cyl_sart_residual.argtypes = [vp, i32, vp, C.c_int, vp, C.c_int, vp, C.c_int, vp,
                                      C.c_size_t, vp]
    lib.cyl_sart_residual.restype = C.c_int
    lib.cyl_sart_update.argtypes = [vp, i32, C.c_double, i32, vp, C.c_int, vp, C.c_int, vp,
                                    C.c_size_t, vp]
    lib.cyl_sart_update.restype = C.c_int
    lib.cyl_sart_batch_step.argtypes = [i32, P(cyl_sart_batch_item), C.c_int, C.c_int, C.c_int,
                                         C.c_int, vp]
    lib.cyl_sart_batch_step.restype = C.c_int
    lib.cyl_fp_diff.argtypes = [vp, vp, C.c_int, vp, C.c_int, vp, C.c_int, i32, i32, vp]
    lib.cyl_fp_diff.restype = C.c_int
    lib.cyl_add.argtypes = [C.c_int64, vp, C.c_int, vp, C.c_int, vp, C.c_int, i32, vp]
    lib.cyl_add.restype = C.c_int
    lib.cyl_axis_corners.argtypes = [i32, i32, i32, vp, C.c_int, C.c_double, i32, vp, i32, vp]
    lib.cyl_axis_corners.restype = C.c_int
    lib.cyl_track_point.argtypes = [P(cyl_traj), P(C.c_double), P(C.c_uint8), P(C.c_double), P(C.c_double)]
    lib.cyl_track_point.restype = C.c_int
    lib.cyl_pose_from_axis.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double, C.c_double,
                                       P(cyl_pose)]
    lib.cyl_pose_from_axis.restype = C.c_int
    lib.cyl_side_sums.argtypes = [i32, i32, i32, vp, C.c_int, vp, vp, vp, vp, i32, vp]
    lib.cyl_side_sums.restype = C.c_int
    lib.cyl_azimuth_phase.argtypes = [i32, P(C.c_double), P(C.c_double), P(C.c_double)]
    lib.cyl_azimuth_phase.restype = C.c_int
    lib.cyl_gamma_from_phase.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, P(C.c_double)]
    lib.cyl_gamma_from_phase.restype = C.c_int
    lib.cyl_axis_points.argtypes = [i32, P(C.c_int32), P(C.c_double), P(C.c_double), P(C.c_uint8)]
    lib.cyl_axis_points.restype = C.c_int
    lib.cyl_mtf.argtypes = [i32, i32, i32, vp, C.c_int, i32, vp, i32, vp]
    lib.cyl_mtf.restype = C.c_int
    lib.cyl_fp_sampled.argtypes = [vp, vp, C.c_int, vp, C.c_int, i32, i32, C.c_double, i32, vp]
    lib.cyl_fp_sampled.restype = C.c_int
    lib.cyl_bp_voxel.argtypes = [vp, vp, C.c_int, vp, C.c_int, i32, i32, i32, vp]
    lib.cyl_bp_voxel.restype = C.c_int
    lib.cyl_sart_run_sampled.argtypes = [vp, P(cyl_sart_params), C.c_double, i32, vp, C.c_int, vp, C.c_int, vp,
                                         C.c_int, vp, C.c_int, vp, C.c_size_t, vp]
    lib.cyl_sart_run_sampled.restype = C.c_int
    lib.cyl_sym_create.argtypes = [vp, P(vp), vp]
    lib.cyl_sym_create.restype = C.c_int
    lib.cyl_sym_destroy.argtypes = [vp]
    lib.cyl_sym_destroy.restype = None
    lib.cyl_sym_nnz.argtypes = [vp]
    lib.cyl_sym_nnz.restype = C.c_int64
    lib.cyl_sym_fp.argtypes = [vp, vp, C.c_int, vp, C.c_int, i32, i32, vp]
    lib.cyl_sym_fp.restype = C.c_int
    lib.cyl_sym_sart_run.argtypes = [vp, P(cyl_sart_params), vp, C.c_int, vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                     vp, C.c_size_t, vp]
    lib.cyl_sym_sart_run.restype = C.c_int
    lib.cyl_last_error.argtypes = []
    lib.cyl_last_error.restype = C.c_char_p
    lib.cyl_version.argtypes = []
    lib.cyl_version.restype = C.c_char_p
    return lib


def lib():
    """The loaded libcyl.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcyl.so not found at %s: build it with "
                               "`python -m paper_2005_11976_amd.build`" % LIB_PATH)
        # torch first: its HIP runtime must be the process's one (libcyl.so
        # then binds to it); loaded the other way round, torch finds no GPU
        import torch  # noqa: F401
        _lib = declare(C.CDLL(LIB_PATH))
    return _lib


def _check(rc, L=None):
    if rc != CYL_OK:
        L = L or lib()
        raise CylError(rc, L.cyl_last_error().decode())


def grid_struct(g):
    return cyl_grid(g.n_h, g.n_theta, g.n_r, g.r_min, g.r_max, g.h_min, g.h_max, g.theta0)


def pose_struct(R, T):
    p = cyl_pose()
    p.R[:] = [float(x) for x in np.asarray(R, dtype=np.float64).ravel()]
    p.T[:] = [float(x) for x in np.asarray(T, dtype=np.float64).ravel()]
    return p


def _dtype_code(t):
    import torch
    codes = {torch.float32: CYL_F32, torch.float16: CYL_F16, torch.bfloat16: CYL_BF16}
    if t.dtype not in codes:
        raise TypeError("unsupported dtype %s (float32, float16, bfloat16)" % t.dtype)
    return codes[t.dtype]


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Geometry:
    """A libcyl geometry (grid, trajectory, pose) resident on one GPU."""

    def __init__(self, scan, device=0, _lib=None):
        self._L = _lib or lib()
        self.scan = scan
        self.device = device
        views = np.ascontiguousarray(scan.views, dtype=np.float64)
        self._views = views
        traj = cyl_traj(scan.n_views, scan.det_rows, scan.det_cols,
                        views.ctypes.data_as(C.POINTER(C.c_double)))
        g = grid_struct(scan.grid)
        pose = pose_struct(scan.R, scan.T)
        h = C.c_void_p()
        _check(self._L.cyl_geom_create(C.byref(g), C.byref(traj), C.byref(pose), device,
                                       C.byref(h)), self._L)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self._L.cyl_geom_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- checks ---------------------------------------------------------------
    def _vol(self, t):
        g = self.scan.grid
        if not (t.is_cuda and t.is_contiguous() and t.numel() == g.n_vox):
            raise ValueError("volume must be a contiguous CUDA tensor with %d elements" % g.n_vox)
        return t

    def _proj(self, t):
        n = self.scan.n_views * self.scan.det_rows * self.scan.det_cols
        if not (t.is_cuda and t.is_contiguous() and t.numel() == n):
            raise ValueError("projections must be a contiguous CUDA tensor with %d elements" % n)
        return t

    # -- entry points -------------------------------------------------------
    def fp(self, vol, proj=None, view_begin=0, view_end=None, out_dtype=None, stream=None):
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        self._vol(vol)
        if proj is None:
            proj = torch.zeros(self.scan.proj_shape, dtype=out_dtype or vol.dtype, device=vol.device)
        self._proj(proj)
        _check(self._L.cyl_fp(self.handle, C.c_void_p(vol.data_ptr()), _dtype_code(vol),
                              C.c_void_p(proj.data_ptr()), _dtype_code(proj), view_begin, view_end,
                              _stream_ptr(stream)), self._L)
        return proj

    def fp_diff(self, vol, base, out=None, view_begin=0, view_end=None, out_dtype=None, stream=None):
        """out = base - A vol (cyl_fp_diff); out defaults to a new tensor of
        base's dtype (or out_dtype)."""
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        self._vol(vol)
        self._proj(base)
        if out is None:
            out = torch.empty(self.scan.proj_shape, dtype=out_dtype or base.dtype, device=base.device)
        self._proj(out)
        _check(self._L.cyl_fp_diff(self.handle, C.c_void_p(vol.data_ptr()), _dtype_code(vol),
                                   C.c_void_p(base.data_ptr()), _dtype_code(base),
                                   C.c_void_p(out.data_ptr()), _dtype_code(out), view_begin, view_end,
                                   _stream_ptr(stream)), self._L)
        return out

    def bp(self, proj, vol=None, view_begin=0, view_end=None, accumulate=False, out_dtype=None,
           stream=None):
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        self._proj(proj)
        if vol is None:
            vol = torch.empty(self.scan.grid.shape, dtype=out_dtype or proj.dtype, device=proj.device)
            accumulate = False
        self._vol(vol)
        _check(self._L.cyl_bp(self.handle, C.c_void_p(proj.data_ptr()), _dtype_code(proj),
                              C.c_void_p(vol.data_ptr()), _dtype_code(vol), view_begin, view_end,
                              int(bool(accumulate)), _stream_ptr(stream)), self._L)
        return vol

    def row_sums(self, out=None, view_begin=0, view_end=None, stream=None):
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        if out is None:
            out = torch.zeros(self.scan.proj_shape, dtype=torch.float32, device="cuda:%d" % self.device)
        self._proj(out)
        if out.dtype != torch.float32:
            raise TypeError("row sums are float32")
        _check(self._L.cyl_row_sums(self.handle, C.c_void_p(out.data_ptr()), view_begin, view_end,
                                    _stream_ptr(stream)), self._L)
        return out

    def sart_params(self, n_iter, lam=0.5, nonneg=False, view_order=None, start_iter=0,
                    start_view=0):
        prm = cyl_sart_params()
        prm.n_iter, prm.lam, prm.nonneg = n_iter, lam, int(bool(nonneg))
        prm.start_iter, prm.start_view = start_iter, start_view
        keep = None
        if view_order is not None:
            keep = np.ascontiguousarray(view_order, dtype=np.int32).ravel()
            if keep.size != self.scan.n_views:
                raise ValueError("view_order needs exactly n_views = %d entries" % self.scan.n_views)
            prm.view_order = keep.ctypes.data_as(C.POINTER(C.c_int32))
        return prm, keep

    def workspace_bytes(self, prm=None):
        prm = prm or self.sart_params(1)[0]
        return int(self._L.cyl_sart_workspace_bytes(self.handle, C.byref(prm)))

    def sart(self, proj, vol, n_iter, lam=0.5, proj_weights=None, vox_weights=None, nonneg=False,
             view_order=None, start_iter=0, start_view=0, workspace=None, stream=None):
        """Weighted SART in place on `vol` (prior in, result out)."""
        import torch
        self._proj(proj)
        self._vol(vol)
        prm, keep = self.sart_params(n_iter, lam, nonneg, view_order, start_iter, start_view)
        need = self.workspace_bytes(prm)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=vol.device)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        if proj_weights is not None:
            self._proj(proj_weights)
        if vox_weights is not None:
            self._vol(vox_weights)
        _check(self._L.cyl_sart_run(
            self.handle, C.byref(prm), C.c_void_p(proj.data_ptr()), _dtype_code(proj),
            pw, _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            vw, _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)
        del keep
        return vol

    def sart_static(self, proj, vol, n_iter, lam=0.5, proj_weights=None, vox_weights=None, nonneg=False,
                    view_order=None, start_iter=0, start_view=0, stream=None):
        """cyl_sart_run_static: weighted SART in place on `vol` with the
        library's static device scratch (no workspace, nothing allocated)."""
        self._proj(proj)
        self._vol(vol)
        prm, keep = self.sart_params(n_iter, lam, nonneg, view_order, start_iter, start_view)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        if proj_weights is not None:
            self._proj(proj_weights)
        if vox_weights is not None:
            self._vol(vox_weights)
        _check(self._L.cyl_sart_run_static(
            self.handle, C.byref(prm), C.c_void_p(proj.data_ptr()), _dtype_code(proj),
            pw, _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            vw, _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), _stream_ptr(stream)), self._L)
        del keep
        return vol

    # -- the paper's own projector pair (comparison) ------------------------
    def fp_sampled(self, vol, step, interp=0, proj=None, view_begin=0, view_end=None, out_dtype=None,
                   stream=None):
        """cyl_fp_sampled: equidistant samples along each ray (interp 0:
        nearest cell, 1: trilinear)."""
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        self._vol(vol)
        if proj is None:
            proj = torch.zeros(self.scan.proj_shape, dtype=out_dtype or vol.dtype, device=vol.device)
        self._proj(proj)
        _check(self._L.cyl_fp_sampled(self.handle, C.c_void_p(vol.data_ptr()), _dtype_code(vol),
                                      C.c_void_p(proj.data_ptr()), _dtype_code(proj), view_begin, view_end,
                                      float(step), int(interp), _stream_ptr(stream)), self._L)
        return proj

    def bp_voxel(self, proj, vol=None, view_begin=0, view_end=None, accumulate=False, out_dtype=None,
                 stream=None):
        """cyl_bp_voxel: voxel-driven bilinear back-projection."""
        import torch
        view_end = self.scan.n_views if view_end is None else view_end
        self._proj(proj)
        if vol is None:
            vol = torch.zeros(self.scan.grid.shape, dtype=out_dtype or proj.dtype, device=proj.device)
        self._vol(vol)
        _check(self._L.cyl_bp_voxel(self.handle, C.c_void_p(proj.data_ptr()), _dtype_code(proj),
                                    C.c_void_p(vol.data_ptr()), _dtype_code(vol), view_begin, view_end,
                                    int(bool(accumulate)), _stream_ptr(stream)), self._L)
        return vol

    def sart_sampled(self, proj, vol, n_iter, step, interp=0, lam=0.5, proj_weights=None, vox_weights=None,
                     nonneg=False, view_order=None, start_iter=0, start_view=0, workspace=None, stream=None):
        """cyl_sart_run_sampled: SART with the paper's sampled FP and
        voxel-driven BP, in place on `vol`."""
        import torch
        self._proj(proj)
        self._vol(vol)
        prm, keep = self.sart_params(n_iter, lam, nonneg, view_order, start_iter, start_view)
        need = self.workspace_bytes(prm)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=vol.device)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        _check(self._L.cyl_sart_run_sampled(
            self.handle, C.byref(prm), float(step), int(interp), C.c_void_p(proj.data_ptr()), _dtype_code(proj),
            pw, _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            vw, _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)
        del keep
        return vol

    def os_workspace_bytes(self, subset):
        return int(self._L.cyl_os_sart_workspace_bytes(self.handle, int(subset)))

    def os_sart(self, proj, vol, n_iter, subset, lam=0.5, proj_weights=None, vox_weights=None, nonneg=False,
                view_order=None, start_iter=0, start_view=0, workspace=None, stream=None):
        """Ordered-subset SART in place on `vol`: `subset` views per update
        (cyl_os_sart_run; subset = n_views is SIRT)."""
        import torch
        self._proj(proj)
        self._vol(vol)
        prm, keep = self.sart_params(n_iter, lam, nonneg, view_order, start_iter, start_view)
        need = self.os_workspace_bytes(subset)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=vol.device)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        if proj_weights is not None:
            self._proj(proj_weights)
        if vox_weights is not None:
            self._vol(vox_weights)
        _check(self._L.cyl_os_sart_run(
            self.handle, C.byref(prm), int(subset), C.c_void_p(proj.data_ptr()), _dtype_code(proj),
            pw, _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            vw, _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)
        del keep
        return vol

    def sart_residual(self, view, proj, vol, workspace, proj_weights=None, stream=None):
        """FP + residual epilogue of one view into `workspace` (FP32 rho)."""
        self._proj(proj)
        self._vol(vol)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        _check(self._L.cyl_sart_residual(
            self.handle, int(view), C.c_void_p(proj.data_ptr()), _dtype_code(proj), pw,
            _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)

    def sart_update(self, view, vol, workspace, lam=0.5, vox_weights=None, nonneg=False,
                    stream=None):
        """BP + weighted update epilogue of one view, in place on `vol`."""
        self._vol(vol)
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        _check(self._L.cyl_sart_update(
            self.handle, int(view), float(lam), int(bool(nonneg)), vw,
            _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)


class BatchEntry:
    """One scan's part of a batched SART sub-iteration (see sart_batch_step)."""

    def __init__(self, geom, view, proj, vol, workspace, proj_weights=None, vox_weights=None,
                 lam=0.5, nonneg=False):
        self.geom, self.view, self.proj, self.vol = geom, int(view), proj, vol
        self.workspace, self.proj_weights, self.vox_weights = workspace, proj_weights, vox_weights
        self.lam, self.nonneg = float(lam), bool(nonneg)


def sart_batch_step(entries, stream=None, _lib=None):
    """cyl_sart_batch_step: one SART sub-iteration (FP + residual, then BP +
    update) for every entry, in two launches for up to 16 entries.  Storage
    types must agree across entries."""
    L = _lib or lib()
    n = len(entries)
    if n == 0:
        return
    arr = (cyl_sart_batch_item * n)()
    e0 = entries[0]
    for i, e in enumerate(entries):
        e.geom._proj(e.proj)
        e.geom._vol(e.vol)
        for t, ref, what in ((e.proj, e0.proj, "projections"), (e.vol, e0.vol, "volumes")):
            if t.dtype != ref.dtype:
                raise TypeError("batch entries must share the %s dtype" % what)
        if e.proj_weights is not None:
            e.geom._proj(e.proj_weights)
        if e.vox_weights is not None:
            e.geom._vol(e.vox_weights)
        a = arr[i]
        a.geom = e.geom.handle.value
        a.view = e.view
        a.proj = e.proj.data_ptr()
        a.proj_weights = e.proj_weights.data_ptr() if e.proj_weights is not None else None
        a.vox_weights = e.vox_weights.data_ptr() if e.vox_weights is not None else None
        a.vol = e.vol.data_ptr()
        a.workspace = e.workspace.data_ptr()
        a.workspace_bytes = e.workspace.numel() * e.workspace.element_size()
        a.lam = e.lam
        a.nonneg = int(e.nonneg)
    pws = [e.proj_weights for e in entries if e.proj_weights is not None]
    vws = [e.vox_weights for e in entries if e.vox_weights is not None]
    if len({t.dtype for t in pws}) > 1 or len({t.dtype for t in vws}) > 1:
        raise TypeError("batch entries must share the weight dtypes")
    pwt = _dtype_code(pws[0]) if pws else CYL_F32
    vwt = _dtype_code(vws[0]) if vws else CYL_F32
    _check(L.cyl_sart_batch_step(n, arr, _dtype_code(e0.proj), pwt, vwt, _dtype_code(e0.vol),
                                 _stream_ptr(stream)), L)


def add(a, b, out=None, stream=None, _lib=None):
    """out = a + b elementwise on the device (cyl_add), FP32 arithmetic."""
    import torch
    L = _lib or lib()
    if a.numel() != b.numel() or not (a.is_cuda and b.is_cuda and a.is_contiguous() and b.is_contiguous()):
        raise ValueError("add needs two contiguous CUDA tensors of equal size")
    if out is None:
        out = torch.empty_like(a)
    if out.numel() != a.numel() or not out.is_contiguous():
        raise ValueError("output size mismatch")
    _check(L.cyl_add(a.numel(), C.c_void_p(a.data_ptr()), _dtype_code(a), C.c_void_p(b.data_ptr()),
                     _dtype_code(b), C.c_void_p(out.data_ptr()), _dtype_code(out), a.device.index or 0,
                     _stream_ptr(stream)), L)
    return out


# -- pose estimation (Sec. 2.1) ------------------------------------------------

def axis_corners(proj, threshold, dilate=1, stream=None, _lib=None):
    """cyl_axis_corners on a [n_views, rows, cols] CUDA tensor: int32 tensor
    [n_views, 9] (four corners (u, v) and the segment's seed-pixel count)."""
    import torch
    L = _lib or lib()
    if proj.dim() != 3 or not (proj.is_cuda and proj.is_contiguous()):
        raise ValueError("projections must be a contiguous CUDA tensor [n_views, rows, cols]")
    n, rows, cols = proj.shape
    out = torch.empty((n, 9), dtype=torch.int32, device=proj.device)
    _check(L.cyl_axis_corners(n, rows, cols, C.c_void_p(proj.data_ptr()), _dtype_code(proj), float(threshold),
                              int(dilate), C.c_void_p(out.data_ptr()), proj.device.index or 0,
                              _stream_ptr(stream)), L)
    return out


def axis_points(corners, _lib=None):
    """cyl_axis_points (host): top and bottom axis points (u, v) per view from
    cyl_axis_corners output ([n, 9] int32), and the mask of views with a
    segment."""
    L = _lib or lib()
    c = np.ascontiguousarray(np.asarray(corners), dtype=np.int32)
    n = c.shape[0]
    top = np.zeros((n, 2))
    bottom = np.zeros((n, 2))
    valid = np.zeros(n, dtype=np.uint8)
    _check(L.cyl_axis_points(n, c.ctypes.data_as(C.POINTER(C.c_int32)), top.ctypes.data_as(C.POINTER(C.c_double)),
                             bottom.ctypes.data_as(C.POINTER(C.c_double)), valid.ctypes.data_as(C.POINTER(C.c_uint8))),
           L)
    return top, bottom, valid.astype(bool)


def gamma_from_phase(phi_p, phi_g, a1, a2, _lib=None):
    """cyl_gamma_from_phase (host): the last Euler angle of Eq. 5."""
    L = _lib or lib()
    out = C.c_double()
    _check(L.cyl_gamma_from_phase(float(phi_p), float(phi_g), float(a1), float(a2), C.byref(out)), L)
    return out.value


def track_point(views, rows, cols, uv, valid=None, _lib=None):
    """cyl_track_point (host): the stage-frame point best matching detector
    points uv [n_views, 2] of views (n_views x 12 stage-frame vectors)."""
    L = _lib or lib()
    v = np.ascontiguousarray(views, dtype=np.float64)
    traj = cyl_traj(v.shape[0], rows, cols, v.ctypes.data_as(C.POINTER(C.c_double)))
    uvc = np.ascontiguousarray(uv, dtype=np.float64)
    if uvc.shape != (v.shape[0], 2):
        raise ValueError("uv must be [n_views, 2]")
    vm = None
    if valid is not None:
        vm = np.ascontiguousarray(valid, dtype=np.uint8)
    xyz = (C.c_double * 3)()
    rms = C.c_double()
    _check(L.cyl_track_point(C.byref(traj), uvc.ctypes.data_as(C.POINTER(C.c_double)),
                             vm.ctypes.data_as(C.POINTER(C.c_uint8)) if vm is not None else None, xyz,
                             C.byref(rms)), L)
    return np.array(xyz[:]), rms.value


def pose_from_axis(top, bottom, h_top, h_bottom, alpha, _lib=None):
    """cyl_pose_from_axis (host): (R, T) of Eq. 1."""
    L = _lib or lib()
    t = (C.c_double * 3)(*[float(x) for x in top])
    b = (C.c_double * 3)(*[float(x) for x in bottom])
    out = cyl_pose()
    _check(L.cyl_pose_from_axis(t, b, float(h_top), float(h_bottom), float(alpha), C.byref(out)), L)
    return np.array(out.R[:]).reshape(3, 3), np.array(out.T[:])


def side_sums(proj, centre, row_lo, row_hi, stream=None, _lib=None):
    """cyl_side_sums on a [n, rows, cols] CUDA tensor; centre, row_lo, row_hi
    host sequences of length n.  Returns a float64 CUDA tensor [n, 2]."""
    import torch
    L = _lib or lib()
    if proj.dim() != 3 or not (proj.is_cuda and proj.is_contiguous()):
        raise ValueError("projections must be a contiguous CUDA tensor [n_views, rows, cols]")
    n, rows, cols = proj.shape
    dev = proj.device
    c = torch.as_tensor(np.asarray(centre, dtype=np.float64).reshape(n), device=dev).contiguous()
    lo = torch.as_tensor(np.asarray(row_lo, dtype=np.int32).reshape(n), device=dev).contiguous()
    hi = torch.as_tensor(np.asarray(row_hi, dtype=np.int32).reshape(n), device=dev).contiguous()
    out = torch.empty((n, 2), dtype=torch.float64, device=dev)
    _check(L.cyl_side_sums(n, rows, cols, C.c_void_p(proj.data_ptr()), _dtype_code(proj),
                           C.c_void_p(c.data_ptr()), C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()),
                           C.c_void_p(out.data_ptr()), dev.index or 0, _stream_ptr(stream)), L)
    return out


class SymMatrix:
    """cyl_sym_*: view 0's exact system matrix, reused for every view of an
    unposed scan whose views are whole-sector rotations of view 0.  Keeps
    its geometry alive."""

    def __init__(self, geom, stream=None):
        self.geom = geom
        self._L = geom._L
        h = C.c_void_p()
        _check(self._L.cyl_sym_create(geom.handle, C.byref(h), _stream_ptr(stream)), self._L)
        self.handle = h

    @property
    def nnz(self):
        return int(self._L.cyl_sym_nnz(self.handle))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self._L.cyl_sym_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fp(self, vol, proj=None, view_begin=0, view_end=None, out_dtype=None, stream=None):
        import torch
        g = self.geom
        view_end = g.scan.n_views if view_end is None else view_end
        g._vol(vol)
        if proj is None:
            proj = torch.zeros(g.scan.proj_shape, dtype=out_dtype or vol.dtype, device=vol.device)
        g._proj(proj)
        _check(self._L.cyl_sym_fp(self.handle, C.c_void_p(vol.data_ptr()), _dtype_code(vol),
                                  C.c_void_p(proj.data_ptr()), _dtype_code(proj), view_begin, view_end,
                                  _stream_ptr(stream)), self._L)
        return proj

    def sart(self, proj, vol, n_iter, lam=0.5, proj_weights=None, vox_weights=None, nonneg=False, view_order=None,
             start_iter=0, start_view=0, workspace=None, stream=None):
        import torch
        g = self.geom
        g._proj(proj)
        g._vol(vol)
        prm, keep = g.sart_params(n_iter, lam, nonneg, view_order, start_iter, start_view)
        need = g.workspace_bytes(prm)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=vol.device)
        pw = C.c_void_p(proj_weights.data_ptr()) if proj_weights is not None else None
        vw = C.c_void_p(vox_weights.data_ptr()) if vox_weights is not None else None
        _check(self._L.cyl_sym_sart_run(
            self.handle, C.byref(prm), C.c_void_p(proj.data_ptr()), _dtype_code(proj),
            pw, _dtype_code(proj_weights) if proj_weights is not None else CYL_F32,
            vw, _dtype_code(vox_weights) if vox_weights is not None else CYL_F32,
            C.c_void_p(vol.data_ptr()), _dtype_code(vol), C.c_void_p(workspace.data_ptr()),
            workspace.numel() * workspace.element_size(), _stream_ptr(stream)), self._L)
        del keep
        return vol


def mtf(vol, window=0, stream=None, _lib=None):
    """cyl_mtf on a contiguous CUDA volume [n_h, n_theta, n_r]: modulation
    (Eq. 8) per ring of the central slice (window 0) or per window of
    `window` rings.  Returns a float64 CUDA tensor."""
    import torch
    L = _lib or lib()
    if vol.dim() != 3 or not (vol.is_cuda and vol.is_contiguous()):
        raise ValueError("volume must be a contiguous CUDA tensor [n_h, n_theta, n_r]")
    nh, nt, nr = vol.shape
    n_out = nr if window == 0 else (nr // window if 0 < window <= nr else 0)
    out = torch.empty(max(n_out, 1), dtype=torch.float64, device=vol.device)
    _check(L.cyl_mtf(nh, nt, nr, C.c_void_p(vol.data_ptr()), _dtype_code(vol), int(window),
                     C.c_void_p(out.data_ptr()), vol.device.index or 0, _stream_ptr(stream)), L)
    return out[:n_out]


def azimuth_phase(s, s_ref, _lib=None):
    """cyl_azimuth_phase (host): internal rotation angle in [0, 2 pi)."""
    L = _lib or lib()
    a = np.ascontiguousarray(s, dtype=np.float64)
    b = np.ascontiguousarray(s_ref, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("signals must be 1-D and of equal length")
    out = C.c_double()
    _check(L.cyl_azimuth_phase(a.size, a.ctypes.data_as(C.POINTER(C.c_double)),
                               b.ctypes.data_as(C.POINTER(C.c_double)), C.byref(out)), L)
    return out.value
