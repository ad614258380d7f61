"""The host half of pose estimation through the C ABI (no GPU needed):
cyl_track_point against the scipy Levenberg-Marquardt of the reference, and
cyl_pose_from_axis against the reference and known poses."""
import numpy as np
import pytest

from oracle import pose as P
from paper_2005_11976_amd import inputs as I


@pytest.fixture(scope="module")
def cyl():
    from paper_2005_11976_amd import cyl as c
    try:
        c.lib()
    except RuntimeError as e:
        pytest.skip(str(e))
    return c


def test_track_point_exact_and_noisy(cyl):
    views = I.circular_views(30, 200.0, 400.0, 0.2, phi0=0.1)
    rng = np.random.default_rng(11)
    for X in (np.array([0.0, 0.0, 0.0]), np.array([5.0, -3.0, 17.0]), np.array([-14.0, 8.0, -22.0])):
        uv = P.project(views, 512, 384, X)
        got, rms = cyl.track_point(views, 512, 384, uv)
        assert np.allclose(got, X, atol=1e-8) and rms < 1e-8
        noisy = uv + rng.normal(scale=0.3, size=uv.shape)
        got, rms = cyl.track_point(views, 512, 384, noisy)
        want, wrms = P.track_point(views, 512, 384, noisy, x0=got)
        assert np.allclose(got, want, atol=1e-7), (got, want)
        assert abs(rms - wrms) <= 1e-9


def test_track_point_valid_mask_and_errors(cyl):
    views = I.circular_views(12, 200.0, 400.0, 0.2)
    uv = P.project(views, 256, 256, np.array([2.0, 1.0, -4.0]))
    valid = np.ones(12, bool)
    valid[::4] = False
    uv[~valid] = np.nan
    got, _ = cyl.track_point(views, 256, 256, uv, valid)
    assert np.allclose(got, [2.0, 1.0, -4.0], atol=1e-8)
    with pytest.raises(cyl.CylError):
        cyl.track_point(views, 256, 256, uv)  # NaN in a valid view
    one = np.zeros(12, bool)
    one[3] = True
    with pytest.raises(cyl.CylError):
        cyl.track_point(views, 256, 256, uv, one)


def test_pose_from_axis_matches_reference_and_truth(cyl):
    for seed in range(5):
        R, T, prm = I.random_pose(2200 + seed, max_tilt_deg=6.0)
        top = R.T @ (np.array([0.0, 0.0, 12.0]) - T)
        bot = R.T @ (np.array([0.0, 0.0, -9.0]) - T)
        R1, T1 = cyl.pose_from_axis(top, bot, 12.0, -9.0, prm["alpha"])
        R2, T2 = P.pose_from_axis(top, bot, 12.0, -9.0, prm["alpha"])
        assert np.allclose(R1, R2, atol=1e-13) and np.allclose(T1, T2, atol=1e-12)
        assert np.allclose(R1, R, atol=1e-12) and np.allclose(T1, T, atol=1e-10)
    with pytest.raises(cyl.CylError):
        cyl.pose_from_axis(top, top, 1.0, 0.0, 0.0)
    with pytest.raises(cyl.CylError):
        cyl.pose_from_axis(top, bot, 0.0, 1.0, 0.0)


def test_azimuth_phase_matches_reference(cyl):
    rng = np.random.default_rng(17)
    for n in (36, 72, 91, 120):
        phi = np.arange(n) * (2 * np.pi / n)
        coef = rng.normal(size=(6, 2))
        def sig(x):
            return sum(c[0] * np.cos((m + 1) * x) + c[1] * np.sin((m + 1) * x) for m, c in enumerate(coef)) + 0.7
        for a in (0.3, 2.2, 4.9):
            s, r = sig(phi + a), sig(phi)
            got = cyl.azimuth_phase(s, r)
            assert abs(got - P.azimuth_phase(s, r)) < 1e-9
            assert abs((got - a + np.pi) % (2 * np.pi) - np.pi) < 1e-8
    with pytest.raises(cyl.CylError):
        cyl.azimuth_phase(np.zeros(2), np.zeros(2))
    with pytest.raises(cyl.CylError):
        cyl.azimuth_phase(np.array([0.0, np.nan, 1.0]), np.zeros(3))
