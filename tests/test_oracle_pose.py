"""Pins of the pose-estimation reference (oracle/pose.py) against facts that do
not come from it: brute-force dilation, rectangle corners, collinearity of
source, pixel and point, exact recovery of known points and poses, and the
axis of a synthetic posed cylinder projected by the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import pose, ref
from paper_2005_11976_amd import inputs as I


def test_segment_matches_brute_force_dilation():
    rng = np.random.default_rng(7)
    for k in (0, 1, 2):
        p = rng.uniform(0, 1, size=(9, 13))
        m = pose.segment(p, 0.93, k)
        seed = p > 0.93
        want = np.zeros_like(seed)
        for v in range(9):
            for u in range(13):
                want[v, u] = seed[max(0, v - k):v + k + 1, max(0, u - k):u + k + 1].any()
        assert np.array_equal(m, want)


def test_corners_of_a_rectangle_and_ties():
    m = np.zeros((20, 30), bool)
    m[4:11, 7:19] = True
    assert pose.corners(m) == [(7, 4), (18, 4), (7, 10), (18, 10)]
    assert pose.corners(np.zeros((3, 3), bool)) is None
    # a diamond: every corner key has a unique extreme pixel
    d = np.zeros((11, 11), bool)
    for v in range(11):
        w = 5 - abs(v - 5)
        d[v, 5 - w:5 + w + 1] = True
    c = pose.corners(d)
    assert c[0] == (5, 0) or c[0][0] + c[0][1] == 5
    # ties on u + v: the topmost pixel wins for the top-left corner
    t = np.zeros((5, 5), bool)
    t[1, 2] = t[2, 1] = t[3, 3] = True
    assert pose.corners(t)[0] == (2, 1)


def test_projection_is_collinear_with_source_and_pixel():
    views = I.circular_views(7, 200.0, 400.0, 0.2, 0.25, phi0=0.3)
    X = np.array([3.0, -7.5, 11.0])
    uv = pose.project(views, 300, 400, X)
    for vw, (u, v) in zip(views, uv):
        S, D, U, V = vw[0:3], vw[3:6], vw[6:9], vw[9:12]
        P = D + (u - 199.5) * U + (v - 149.5) * V
        c = np.cross(P - S, X - S)
        assert np.linalg.norm(c) <= 1e-9 * np.linalg.norm(P - S) * np.linalg.norm(X - S)


def test_track_point_recovers_known_points():
    views = I.circular_views(24, 200.0, 400.0, 0.2)
    for X in (np.array([0.0, 0.0, 0.0]), np.array([4.0, -2.0, 19.0]), np.array([-12.0, 9.0, -21.0])):
        uv = pose.project(views, 512, 512, X)
        got, rms = pose.track_point(views, 512, 512, uv)
        assert np.allclose(got, X, atol=1e-8) and rms < 1e-8
    valid = np.arange(24) % 3 != 0
    uv = pose.project(views, 512, 512, np.array([1.0, 2.0, 3.0]))
    uv[~valid] = 1e6  # ignored
    got, _ = pose.track_point(views, 512, 512, uv, valid)
    assert np.allclose(got, [1.0, 2.0, 3.0], atol=1e-8)


def test_pose_from_axis_round_trip():
    for seed in range(6):
        R, T, prm = I.random_pose(2100 + seed, max_tilt_deg=8.0)
        if prm["beta"] < 1e-3:
            continue
        pts = {h: R.T @ (np.array([0.0, 0.0, h]) - T) for h in (-20.0, 15.0)}
        R2, T2 = pose.pose_from_axis(pts[15.0], pts[-20.0], 15.0, -20.0, prm["alpha"])
        assert np.allclose(R2, R, atol=1e-12) and np.allclose(T2, T, atol=1e-10)


def test_axis_of_a_posed_cylinder_from_oracle_projections():
    """A solid cylinder (r <= 6.25 mm, h in [-6.7, 6.7] mm) under a known pose,
    projected by the FP64 oracle: the tracked axis is within 0.4 deg and
    0.1 mm of the true one.  The silhouette corners are rim points of the caps,
    not their centres, so the tracked axis points carry a perspective bias of
    about r^2 / SOD (0.2 mm here), part of it across the axis."""
    g = I.Grid(18, 64, 16, 0.0, 10.0, -10.0, 10.0)
    R, T = I.pose_from(0.7, math.radians(4.0), 1.9, [0.8, -0.5, 0.6])
    views = I.circular_views(36, 200.0, 400.0, 0.2)
    scan = I.Scan(g, views, 200, 200, R, T)
    vol = np.zeros(g.shape)
    vol[3:15, :, :10] = 0.02  # h in [-6.7, 6.7] mm, r <= 6.25 mm: the silhouette stays on the detector
    p = ref.Oracle(scan).fp(vol)
    pts = pose.axis_points(p, 0.02, 1)
    assert all(x is not None for x in pts)
    for x in pts:
        assert min(c[0] for c in x[2]) > 2 and max(c[0] for c in x[2]) < 197
        assert min(c[1] for c in x[2]) > 2 and max(c[1] for c in x[2]) < 197
    top, _ = pose.track_point(views, 200, 200, [x[0] for x in pts])
    bot, _ = pose.track_point(views, 200, 200, [x[1] for x in pts])
    d_true = R.T @ np.array([0.0, 0.0, 1.0])
    d = (bot - top) / np.linalg.norm(bot - top)  # detector rows grow downwards: "top" is high z
    if d @ d_true < 0:
        d = -d
    ang = math.degrees(math.acos(min(1.0, abs(float(d @ d_true)))))
    centre_true = -R.T @ T
    mid = 0.5 * (top + bot)
    off = (mid - centre_true) - ((mid - centre_true) @ d_true) * d_true
    assert ang < 0.4, ang
    assert np.linalg.norm(off) < 0.1, off


def test_azimuth_phase_of_a_shifted_signal():
    """A band-limited periodic signal sampled at 72 equally spaced view angles
    and its copy advanced by a known angle: the phase is recovered exactly (to
    rounding), whatever the shift between samples."""
    phi = np.arange(72) * (2 * np.pi / 72) + 0.2
    def sig(x):
        return 0.3 + np.cos(x) + 0.4 * np.sin(2 * x + 0.3) + 0.2 * np.cos(3 * x - 1.0)
    for a in (0.0, 0.7, 2.9, 5.5, 0.0123):
        got = pose.azimuth_phase(sig(phi + a), sig(phi))
        err = (got - a + np.pi) % (2 * np.pi) - np.pi
        assert abs(err) < 1e-9, (a, got)


def test_side_sums_by_loops():
    rng = np.random.default_rng(3)
    p = rng.uniform(size=(2, 7, 9))
    out = pose.side_sums(p, [3.5, 4.25], [1, 0], [5, 9])
    for k, (c, a, b) in enumerate(((3.5, 1, 5), (4.25, 0, 6))):
        left = right = 0.0
        for v in range(a, b + 1):
            for u in range(9):
                f = min(1.0, max(0.0, c - (u - 0.5)))
                left += f * p[k, v, u]
                right += (1.0 - f) * p[k, v, u]
        assert np.isclose(out[k, 0], left) and np.isclose(out[k, 1], right)
    # a profile symmetric about its centre splits evenly wherever the centre falls
    for c in (20.0, 20.3, 20.5):
        x = np.arange(41)
        prof = np.exp(-0.02 * (x - c) ** 2)
        img = np.tile(prof, (3, 1))[None]
        ls, rs = pose.side_sums(img, [c], [0], [2])[0]
        assert abs(ls - rs) < 1e-2 * (ls + rs)


def test_internal_rotation_from_oracle_projections():
    """A part with two off-axis inclusions (the azimuthal structure) rotated about
    its axis by a known angle, tilted and shifted; projected by the FP64
    oracle with and without the internal rotation (the reference uses the same
    axis pose): the phase of the grey values beside the projected axis gives
    the internal rotation to within 1.5 degrees."""
    g = I.Grid(24, 96, 16, 0.0, 25.0, -25.0, 25.0)
    vol = np.zeros(g.shape)
    vol[2:22, :, :14] = 0.01       # the part: a cylinder r <= 21.9 mm
    vol[6:18, 8:20, 9:13] = 0.03   # two off-axis inclusions (ring sectors)
    vol[4:9, 50:58, 5:8] = 0.025
    views = I.circular_views(90, 200.0, 400.0, 0.8)
    beta, gamma, centre = math.radians(3.0), 1.2, [0.9, -0.6, 0.4]
    rows = cols = 128
    sig = {}
    for name, alpha in (("ref", 0.0), ("meas", 2.1)):
        R, T = I.pose_from(alpha, beta, gamma, centre)
        scan = I.Scan(g, views, rows, cols, R, T)
        p = ref.Oracle(scan).fp(vol)
        ax = pose.project(views, rows, cols, -R.T @ T)  # projected object origin per view
        ss = pose.side_sums(p, ax[:, 0], np.zeros(90), np.full(90, rows - 1))
        sig[name] = ss[:, 1] - ss[:, 0]
    got = pose.azimuth_phase(sig["meas"], sig["ref"])
    err = math.degrees((got - 2.1 + math.pi) % (2 * math.pi) - math.pi)
    assert abs(err) < 1.5, (got, err)
