"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/cyl.h declares, and rejects invalid arguments with
CYL_EINVAL before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2005_11976_amd import cyl, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cyl.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(cyl.LIB_PATH):
        from paper_2005_11976_amd import build
        build.build()
    return cyl.lib()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cyl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = _declared()
    for n in ["cyl_geom_create", "cyl_geom_destroy", "cyl_fp", "cyl_bp", "cyl_sart_run",
              "cyl_sart_workspace_bytes", "cyl_last_error", "cyl_row_sums", "cyl_version"]:
        assert n in names
    assert set(names) == set(cyl.EXPORTS)


def test_static_scratch_size_matches_header():
    m = re.search(r"#define CYL_SART_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) == cyl.SART_STATIC_SCRATCH_BYTES


def test_library_exports_every_declared_symbol(L):
    for n in _declared():
        assert hasattr(L, n), n
    assert L.cyl_version().decode().startswith("libcyl")
    assert L.cyl_last_error() is not None


def _create(L, grid, views, rows=8, cols=8, R=None, T=None):
    g = cyl.grid_struct(grid)
    v = np.ascontiguousarray(views, dtype=np.float64)
    traj = cyl.cyl_traj(v.shape[0], rows, cols, v.ctypes.data_as(C.POINTER(C.c_double)))
    pose = cyl.pose_struct(np.eye(3) if R is None else R, np.zeros(3) if T is None else T)
    h = C.c_void_p()
    rc = L.cyl_geom_create(C.byref(g), C.byref(traj), C.byref(pose), 0, C.byref(h))
    return rc, h


GOOD = I.Grid(4, 8, 4, 0.0, 5.0, -5.0, 5.0)
VIEWS = I.circular_views(3, 50.0, 100.0, 0.5)


@pytest.mark.parametrize("grid", [
    I.Grid(0, 8, 4, 0.0, 5.0, -5.0, 5.0),
    I.Grid(4, 0, 4, 0.0, 5.0, -5.0, 5.0),
    I.Grid(4, 8, 0, 0.0, 5.0, -5.0, 5.0),
    I.Grid(4, 8, 4, -1.0, 5.0, -5.0, 5.0),
    I.Grid(4, 8, 4, 5.0, 5.0, -5.0, 5.0),
    I.Grid(4, 8, 4, 0.0, 5.0, 5.0, 5.0),
    I.Grid(4, 8, 4, 0.0, float("nan"), -5.0, 5.0),
])
def test_invalid_grid_rejected(L, grid):
    rc, h = _create(L, grid, VIEWS)
    assert rc == cyl.CYL_EINVAL
    assert not h.value
    assert L.cyl_last_error().decode().startswith("cyl_geom_create")


def test_invalid_pose_and_trajectory_rejected(L):
    rc, _ = _create(L, GOOD, VIEWS, R=np.diag([1.0, 1.0, -1.0]))
    assert rc == cyl.CYL_EINVAL and b"reflection" in L.cyl_last_error()
    rc, _ = _create(L, GOOD, VIEWS, R=np.diag([1.0, 2.0, 1.0]))
    assert rc == cyl.CYL_EINVAL and b"orthonormal" in L.cyl_last_error()
    rc, _ = _create(L, GOOD, VIEWS, rows=0)
    assert rc == cyl.CYL_EINVAL
    bad = VIEWS.copy()
    bad[1, 0:3] = [0.5, 0.0, 0.0]  # source inside the support
    rc, _ = _create(L, GOOD, bad)
    assert rc == cyl.CYL_EINVAL and b"inside the grid support" in L.cyl_last_error()
    bad = VIEWS.copy()
    bad[2, 9:12] = bad[2, 6:9]  # u and v steps parallel
    rc, _ = _create(L, GOOD, bad)
    assert rc == cyl.CYL_EINVAL and b"degenerate detector" in L.cyl_last_error()
    bad = VIEWS.copy()
    bad[0, 4] = float("inf")
    rc, _ = _create(L, GOOD, bad)
    assert rc == cyl.CYL_EINVAL


def test_null_arguments_rejected(L):
    assert L.cyl_fp(None, None, 0, None, 0, 0, 1, None) == cyl.CYL_EINVAL
    assert L.cyl_bp(None, None, 0, None, 0, 0, 1, 0, None) == cyl.CYL_EINVAL
    assert L.cyl_row_sums(None, None, 0, 1, None) == cyl.CYL_EINVAL
    assert L.cyl_sart_run(None, None, None, 0, None, 0, None, 0, None, 0, None, 0, None) == cyl.CYL_EINVAL
    assert L.cyl_sart_workspace_bytes(None, None) == 0
    assert L.cyl_sart_run_static(None, None, None, 0, None, 0, None, 0, None, 0, None) == cyl.CYL_EINVAL
    L.cyl_geom_destroy(None)
    g = cyl.grid_struct(GOOD)
    assert L.cyl_geom_create(C.byref(g), None, None, 0, None) == cyl.CYL_EINVAL


def test_error_message_is_thread_local(L):
    import threading
    assert L.cyl_fp(None, None, 0, None, 0, 0, 1, None) == cyl.CYL_EINVAL
    seen = {}

    def other():
        seen["msg"] = L.cyl_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == b""
    assert L.cyl_last_error() != b""


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(cyl, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cyl, "_lib", None)
    with pytest.raises(RuntimeError, match="libcyl.so not found"):
        cyl.lib()
