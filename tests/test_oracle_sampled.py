"""Pins of the reference of the paper's own projector pair (oracle/sampled.py,
Sec. 2.2) against facts that do not come from it:

* the nearest-sample projection converges to the exact line integrals of the
  FP64 oracle as the step shrinks, and its row sums are the support chord to
  within two steps;
* trilinear interpolation reproduces a volume that is linear in the ring
  index (closed form in the sample radius, clamped outside the ring centres);
* the voxel-driven back-projection of an all-ones image counts the views at
  interior cells, and that of a one-pixel image equals the bilinear weight
  of the pixel at the cell centre's projection found by intersecting the
  source-centre line with the detector plane (no matrix solve);
* SART with the pair on one voxel follows mu* + (1 - lam)^K (mu0 - mu*).
"""
import math

import numpy as np
import pytest

from oracle import ref, sampled
from paper_2005_11976_amd import inputs as I


def _scan(grid=None, n_views=4, rows=10, cols=14, posed=False, pitch=0.8):
    grid = grid or I.Grid(4, 12, 5, 0.0, 5.0, -2.0, 2.0, 0.1)
    views = I.circular_views(n_views, 40.0, 80.0, pitch, phi0=0.2)
    R, T = I.pose_from(0.3, 0.2, 0.9, [0.3, -0.2, 0.1]) if posed else I.identity_pose()
    return I.Scan(grid, np.asarray(views, dtype=np.float64), rows, cols, R, T)


@pytest.mark.parametrize("posed", [False, True])
def test_nearest_samples_converge_to_the_exact_projection(posed):
    scan = _scan(posed=posed)
    rng = np.random.default_rng(4700)
    vol = rng.uniform(0.0, 1.0, size=scan.grid.shape)
    exact = ref.Oracle(scan).fp(vol)
    errs = []
    for step in (0.2, 0.05, 0.0125):
        q, _ = sampled.sampled_fp(scan, vol, step, "nearest")
        errs.append(np.linalg.norm(q - exact) / np.linalg.norm(exact))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.01


def test_row_sums_are_the_support_chord_within_two_steps():
    grid = I.Grid(3, 8, 4, 1.0, 5.0, -2.0, 2.0)  # hollow: up to two support pieces
    scan = _scan(grid)
    step = 0.13
    q, L = sampled.sampled_fp(scan, np.ones(grid.shape), step, "nearest")
    np.testing.assert_array_equal(q, L)
    chord = ref.Oracle(scan).row_sums()
    assert np.abs(L - chord).max() <= 2 * step + 1e-12
    assert np.abs(L - chord).max() > 0.01  # the sampling is visible
    q2, _ = sampled.sampled_fp(scan, np.ones(grid.shape), step, "linear")
    np.testing.assert_allclose(q2, L, rtol=1e-13, atol=1e-13)


def test_linear_interpolation_reproduces_a_ring_ramp():
    grid = I.Grid(3, 10, 6, 0.5, 5.0, -2.0, 2.0, 0.3)
    scan = _scan(grid)
    a, b, step = 0.2, 0.05, 0.1
    vol = np.broadcast_to((a + b * np.arange(6))[None, None, :], grid.shape).copy()
    q, _ = sampled.sampled_fp(scan, vol, step, "linear")
    dr = (grid.r_max - grid.r_min) / grid.n_r
    o = ref.Oracle(scan)
    for k, v, u in ((0, 4, 6), (1, 5, 3), (2, 2, 9), (3, 7, 7)):
        ea, ee = o.ray_ends(k, v, u)
        d = ee - ea
        length = np.linalg.norm(d)
        want = 0.0
        for i in range(int(length / step) + 1):
            dist = (i + 0.5) * step
            if dist >= length:
                break
            x = ea + d * (dist / length)
            r = math.hypot(x[0], x[1])
            if not (grid.r_min <= r < grid.r_max and grid.h_min <= x[2] < grid.h_max):
                continue
            fr = min(max((r - grid.r_min) / dr - 0.5, 0.0), grid.n_r - 1.0)
            want += step * (a + b * fr)
        assert q[k, v, u] == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_voxel_bp_counts_views_and_reads_bilinear_weights():
    grid = I.Grid(3, 8, 4, 0.0, 3.0, -1.0, 1.0)
    scan = _scan(grid, n_views=5, rows=12, cols=16, posed=True)
    c, n = sampled.voxel_bp(scan, np.ones((5, 12, 16)))
    np.testing.assert_allclose(c, 5.0, rtol=0, atol=1e-12)  # the grid projects inside every view
    np.testing.assert_allclose(n, 5.0, rtol=0, atol=1e-12)
    # one lit pixel in view 2
    y = np.zeros((1, 12, 16))
    us, vs = 7, 5
    y[0, vs, us] = 1.0
    c1, _ = sampled.voxel_bp(scan, y, 2, 3)
    R, T = np.asarray(scan.R), np.asarray(scan.T)
    w = scan.views[2]
    a = R @ w[0:3] + T
    U, V = R @ w[6:9], R @ w[9:12]
    P0 = R @ (w[3:6] - 7.5 * w[6:9] - 5.5 * w[9:12]) + T
    nrm = np.cross(U, V)
    x = sampled.cell_centres(grid)
    want = np.zeros(len(x))
    for i, xc in enumerate(x):
        t = (P0 - a) @ nrm / ((xc - a) @ nrm)
        P = a + t * (xc - a)
        u = (P - P0) @ U / (U @ U)
        v = (P - P0) @ V / (V @ V)
        want[i] = max(0.0, 1 - abs(u - us)) * max(0.0, 1 - abs(v - vs))
    np.testing.assert_allclose(c1.ravel(), want, rtol=0, atol=1e-12)
    assert want.max() > 0.3


def test_sampled_sart_single_voxel_closed_form():
    grid = I.Grid(1, 1, 1, 0.0, 4.0, -3.0, 3.0)
    views = I.circular_views(3, 30.0, 60.0, 0.5)
    scan = I.Scan(grid, np.asarray(views, dtype=np.float64), 28, 28, *I.identity_pose())
    step, mu_star, mu0, lam = 0.05, 0.03, 0.005, 0.4
    p, _ = sampled.sampled_fp(scan, np.full(grid.shape, mu_star), step, "nearest")
    # the one cell's centre (r = 2, theta = pi, h = 0) lies inside the voxel, so
    # in every view its projection and its four neighbouring pixels see the voxel
    for k in range(3):
        u, v, front = sampled.project_points(sampled._object_views(scan)[k], sampled.cell_centres(grid))
        u0, v0 = int(np.floor(u[0])), int(np.floor(v[0]))
        assert front[0] and (p[k, v0:v0 + 2, u0:u0 + 2] > 0).all()
    for n_iter in (1, 2):
        mu = sampled.sampled_sart(scan, p, np.full(grid.shape, mu0), n_iter, step, "nearest", lam)
        K = 3 * n_iter
        assert mu.ravel()[0] == pytest.approx(mu_star + (1 - lam) ** K * (mu0 - mu_star), rel=1e-12)
