"""Eq. 5 (Sec. 2.1) and the axis points of the corner output, on the host
(no GPU): the oracle's closed form against cases with an independent meaning,
and the C ABI against the oracle."""
import math

import numpy as np
import pytest

from oracle import pose as P


def _wrap(x):
    return x - 2.0 * math.pi * math.floor(x / (2.0 * math.pi))


def test_eq5_untilted_is_a_composition_of_rotations_about_one_axis():
    # beta = 0: the first and last rotations are about the same axis, so the
    # perceived phase is their sum plus the scanner's angle
    for a1 in (-1.2, -0.3, 0.0, 0.4, 1.4):
        for g in (0.1, 2.5, 5.9):
            phi_g = 0.37
            phi_p = g + a1 + phi_g
            assert P.gamma_eq5(phi_p, phi_g, a1, 0.0) == pytest.approx(_wrap(g), abs=1e-12)


def test_eq5_no_first_rotation_needs_no_correction():
    for b in (0.0, 0.2, -0.7, 1.3):
        assert P.gamma_eq5(1.1, 0.25, 0.0, b) == pytest.approx(0.85, abs=1e-12)


def test_eq5_correction_is_the_angle_in_the_tilted_plane():
    # a stage direction at azimuth a1 meets the plane tilted by a2 about the x
    # axis at the in-plane angle whose tangent is tan(a1) / cos(a2): take the
    # in-plane unit vector at angle psi, tilt it, and read its stage azimuth
    for a2 in (0.1, 0.5, 1.0):
        for psi in (-1.3, -0.4, 0.3, 1.2):
            d = np.array([math.cos(psi), math.sin(psi) * math.cos(a2), math.sin(psi) * math.sin(a2)])
            a1 = math.atan2(d[1], d[0])           # its azimuth in the stage frame
            # Eq. 5 with phi_p = phi_g = 0 returns -correction; the correction is psi
            assert _wrap(-P.gamma_eq5(0.0, 0.0, a1, a2)) == pytest.approx(_wrap(psi), abs=1e-12)


def test_eq5_continuous_through_a_quarter_turn():
    for a2 in (0.3, 1.1):
        lo = P.gamma_eq5(0.0, 0.0, math.pi / 2 - 1e-9, a2)
        hi = P.gamma_eq5(0.0, 0.0, math.pi / 2 + 1e-9, a2)
        assert abs(lo - hi) < 1e-6
        assert P.gamma_eq5(0.0, 0.0, math.pi / 2, a2) == pytest.approx(_wrap(-math.pi / 2), abs=1e-12)


@pytest.fixture(scope="module")
def cyl():
    from paper_2005_11976_amd import cyl as c
    try:
        c.lib()
    except RuntimeError as e:
        pytest.skip(str(e))
    return c


def test_gamma_from_phase_abi_matches_oracle(cyl):
    rng = np.random.default_rng(77)
    for _ in range(200):
        phi_p, phi_g = rng.uniform(-7, 7, size=2)
        a1, a2 = rng.uniform(-3, 3), rng.uniform(-1.4, 1.4)
        assert cyl.gamma_from_phase(phi_p, phi_g, a1, a2) == pytest.approx(P.gamma_eq5(phi_p, phi_g, a1, a2),
                                                                           abs=1e-12)
    with pytest.raises(cyl.CylError):
        cyl.gamma_from_phase(float("nan"), 0.0, 0.0, 0.0)


def test_axis_points_abi(cyl):
    c = np.array([[10, 20, 30, 22, 12, 80, 28, 84, 500],
                  [-1, -1, -1, -1, -1, -1, -1, -1, 0],
                  [5, 5, 6, 5, 5, 9, 6, 9, 12]], dtype=np.int32)
    top, bottom, valid = cyl.axis_points(c)
    assert valid.tolist() == [True, False, True]
    assert np.array_equal(top[[0, 2]], [[20.0, 21.0], [5.5, 5.0]])
    assert np.array_equal(bottom[[0, 2]], [[20.0, 82.0], [5.5, 9.0]])
    assert np.all(top[1] == -1.0) and np.all(bottom[1] == -1.0)
