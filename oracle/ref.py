"""ctypes front end of the FP64 CPU oracle (cyl_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cyl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile cyl_oracle.c into liboracle.so with gcc (plain C, FP64, -O2)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
                           "-ffp-contract=off", "-o", tmp, _SRC, "-lm", "-lpthread"])
    os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("n_h", C.c_int32), ("n_theta", C.c_int32), ("n_r", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("h_min", C.c_double),
                ("h_max", C.c_double), ("theta0", C.c_double)]


class _Scan(C.Structure):
    _fields_ = [("g", _Grid), ("n_views", C.c_int32), ("det_rows", C.c_int32),
                ("det_cols", C.c_int32), ("views", C.POINTER(C.c_double)),
                ("R", C.c_double * 9), ("T", C.c_double * 3)]


class _SartParams(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("lam", C.c_double), ("nonneg", C.c_int32),
                ("view_order", C.POINTER(C.c_int32)), ("start_iter", C.c_int32),
                ("start_view", C.c_int32), ("subset", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.POINTER(C.c_double)
        i64 = C.POINTER(C.c_int64)
        _lib.orc_fp.argtypes = [C.POINTER(_Scan), d, C.c_int, C.c_int, d, d, C.c_int]
        _lib.orc_fp_rays.argtypes = [C.POINTER(_Scan), d, C.c_int, i64, C.c_int64, d, d, C.c_int]
        _lib.orc_bp.argtypes = [C.POINTER(_Scan), d, C.c_int, C.c_int, d, d, C.c_int]
        _lib.orc_sart.argtypes = [C.POINTER(_Scan), C.POINTER(_SartParams), d, d, d, d, d,
                                  C.c_int]
        _lib.orc_sart.restype = C.c_int
        _lib.orc_build_csr.argtypes = [C.POINTER(_Scan), C.c_int, C.c_int, i64, i64, d]
        _lib.orc_build_csr.restype = C.c_int64
        _lib.orc_ray_pieces.argtypes = [C.POINTER(_Grid), d, d, i64, d]
        _lib.orc_ray_pieces.restype = C.c_int
        _lib.orc_max_pieces.argtypes = [C.POINTER(_Grid)]
        _lib.orc_max_pieces.restype = C.c_int
        _lib.orc_ray_ends.argtypes = [C.POINTER(_Scan), C.c_int, C.c_int, C.c_int, d, d]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _nthreads(n):
    if n is not None:
        return int(n)
    return max(1, min(16, os.cpu_count() or 1))


def _grid(g):
    return _Grid(g.n_h, g.n_theta, g.n_r, g.r_min, g.r_max, g.h_min, g.h_max, g.theta0)


class Oracle:
    """FP64 oracle bound to one scan (grid, stage-frame views, pose)."""

    def __init__(self, scan):
        self.scan = scan
        self._views = _f64(scan.views)
        st = _Scan()
        st.g = _grid(scan.grid)
        st.n_views, st.det_rows, st.det_cols = scan.n_views, scan.det_rows, scan.det_cols
        st.views = _dp(self._views)
        st.R[:] = [float(x) for x in np.asarray(scan.R, dtype=np.float64).ravel()]
        st.T[:] = [float(x) for x in np.asarray(scan.T, dtype=np.float64).ravel()]
        self._st = st
        self.V = scan.grid.n_vox
        self.P = scan.det_rows * scan.det_cols

    # -- projectors ---------------------------------------------------------
    def fp(self, vol, vb=0, ve=None, nthreads=None, rowsum=False):
        ve = self.scan.n_views if ve is None else ve
        x = _f64(vol).ravel()
        assert x.size == self.V
        q = np.zeros((ve - vb) * self.P)
        L = np.zeros_like(q) if rowsum else None
        lib().orc_fp(C.byref(self._st), _dp(x), vb, ve, _dp(q),
                     _dp(L) if rowsum else None, _nthreads(nthreads))
        shape = (ve - vb, self.scan.det_rows, self.scan.det_cols)
        return (q.reshape(shape), L.reshape(shape)) if rowsum else q.reshape(shape)

    def fp_rays(self, vol, rays, vb=0, nthreads=None):
        """FP (and row sums) of an explicit list of flat ray indices, counted from view vb."""
        x = _f64(vol).ravel()
        r = np.ascontiguousarray(rays, dtype=np.int64)
        q = np.zeros(r.size)
        L = np.zeros(r.size)
        lib().orc_fp_rays(C.byref(self._st), _dp(x), vb,
                          r.ctypes.data_as(C.POINTER(C.c_int64)), r.size, _dp(q), _dp(L),
                          _nthreads(nthreads))
        return q, L

    def row_sums(self, vb=0, ve=None, nthreads=None):
        return self.fp(np.zeros(self.V), vb, ve, nthreads, rowsum=True)[1]

    def bp(self, y, vb=0, ve=None, nthreads=None, colsum=False):
        ve = self.scan.n_views if ve is None else ve
        yy = _f64(y).ravel()
        assert yy.size == (ve - vb) * self.P
        out = np.zeros(self.V)
        cs = np.zeros(self.V) if colsum else None
        lib().orc_bp(C.byref(self._st), _dp(yy), vb, ve, _dp(out), _dp(cs) if colsum else None,
                     _nthreads(nthreads))
        shape = self.scan.grid.shape
        return (out.reshape(shape), cs.reshape(shape)) if colsum else out.reshape(shape)

    # -- SART -----------------------------------------------------------------
    def sart(self, proj, vol0, n_iter, lam=0.5, proj_weights=None, vox_weights=None,
             nonneg=False, view_order=None, start_iter=0, start_view=0, nthreads=None, subset=1):
        """Weighted SART (Eq. 7) with ordered subsets of `subset` projections
        (1: one projection per update, the paper's setting; n_views: SIRT)."""
        p = _f64(proj).ravel()
        assert p.size == self.scan.n_views * self.P
        vol = _f64(vol0).ravel().copy()
        pw = None if proj_weights is None else _f64(proj_weights).ravel()
        vw = None if vox_weights is None else _f64(vox_weights).ravel()
        prm = _SartParams()
        prm.n_iter, prm.lam, prm.nonneg = n_iter, lam, int(bool(nonneg))
        order = None
        if view_order is not None:
            order = np.ascontiguousarray(view_order, dtype=np.int32)
            prm.view_order = order.ctypes.data_as(C.POINTER(C.c_int32))
        prm.start_iter, prm.start_view = start_iter, start_view
        prm.subset = int(subset)
        resid = np.zeros(max(n_iter, 1))
        rc = lib().orc_sart(C.byref(self._st), C.byref(prm), _dp(p),
                            _dp(pw) if pw is not None else None,
                            _dp(vw) if vw is not None else None, _dp(vol), _dp(resid),
                            _nthreads(nthreads))
        if rc != 0:
            raise MemoryError("oracle SART allocation failed")
        return vol.reshape(self.scan.grid.shape), resid[:n_iter]

    # -- explicit matrix (small sizes only) ---------------------------------
    def csr(self, vb=0, ve=None):
        """Rows of A for views [vb, ve) as (indptr, cells, lens)."""
        ve = self.scan.n_views if ve is None else ve
        n = (ve - vb) * self.P
        indptr = np.zeros(n + 1, dtype=np.int64)
        nnz = lib().orc_build_csr(C.byref(self._st), vb, ve,
                                  indptr.ctypes.data_as(C.POINTER(C.c_int64)), None, None)
        cells = np.zeros(nnz, dtype=np.int64)
        lens = np.zeros(nnz)
        lib().orc_build_csr(C.byref(self._st), vb, ve,
                            indptr.ctypes.data_as(C.POINTER(C.c_int64)),
                            cells.ctypes.data_as(C.POINTER(C.c_int64)), _dp(lens))
        return indptr, cells, lens

    def dense(self, vb=0, ve=None):
        """A as a dense (rays, voxels) matrix; tiny grids only."""
        indptr, cells, lens = self.csr(vb, ve)
        n = indptr.size - 1
        A = np.zeros((n, self.V))
        rows = np.repeat(np.arange(n), np.diff(indptr))
        np.add.at(A, (rows, cells), lens)
        return A

    def ray_ends(self, k, v, u):
        a = np.zeros(3)
        e = np.zeros(3)
        lib().orc_ray_ends(C.byref(self._st), k, v, u, _dp(a), _dp(e))
        return a, e


def ray_pieces(grid, a, e):
    """(cells, lengths) of the segment a -> e (object frame) on `grid`."""
    g = _grid(grid)
    cap = lib().orc_max_pieces(C.byref(g))
    cells = np.zeros(cap, dtype=np.int64)
    lens = np.zeros(cap)
    aa, ee = _f64(a), _f64(e)
    n = lib().orc_ray_pieces(C.byref(g), _dp(aa), _dp(ee),
                             cells.ctypes.data_as(C.POINTER(C.c_int64)), _dp(lens))
    return cells[:n].copy(), lens[:n].copy()
