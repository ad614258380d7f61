"""Pins of the MTF reference (oracle/mtf.py, Sec. 2.3 Eq. 8) against closed
forms and explicit loops: the modulation of a + b cos is b / a, a constant has
none, a line phantom whose samples reach both extremes has modulation 1 in
every ring and every one-period window, the central slice of an even stack is
the mean of the two middle slices, and the windowed radial MTF equals
explicit loops over a random volume."""
import math

import numpy as np
import pytest

from oracle import mtf
from paper_2005_11976_amd import inputs as I


def test_modulation_closed_forms():
    for a, b in ((1.0, 0.5), (0.3, 0.3), (2.0, 0.01)):
        x = a + b * np.cos(np.linspace(0.0, 2 * math.pi, 17))  # reaches cos = 1 and cos = -1
        assert mtf.modulation(x) == pytest.approx(b / a, rel=1e-14)
    assert mtf.modulation(np.full(5, 0.7)) == 0.0
    assert mtf.modulation(np.zeros(4)) == 0.0
    assert mtf.modulation([0.0, 2.0]) == 1.0


def test_central_slice_even_and_odd():
    v = np.arange(4 * 3 * 2, dtype=np.float64).reshape(4, 3, 2)
    np.testing.assert_array_equal(mtf.central_slice(v), 0.5 * (v[1] + v[2]))
    w = v[:3]
    np.testing.assert_array_equal(mtf.central_slice(w), w[1])


@pytest.mark.parametrize("n_l", [1, 2, 4, 8, 16])
def test_line_phantoms_have_full_modulation(n_l):
    g = I.Grid(4, 64, 32, 0.0, 10.0, -1.0, 1.0)
    az = I.line_phantom(g, "azimuthal", n_l)
    np.testing.assert_allclose(mtf.mtf_azimuthal(az), 1.0, rtol=0, atol=1e-15)
    rad = I.line_phantom(g, "radial", n_l)
    w = 32 // n_l
    np.testing.assert_allclose(mtf.mtf_radial(rad, w), 1.0, rtol=0, atol=1e-15)
    assert mtf.mtf_slice(az) == pytest.approx(1.0, abs=1e-15)
    # the radial phantom has no azimuthal modulation, the azimuthal one no radial
    np.testing.assert_array_equal(mtf.mtf_azimuthal(rad), 0.0)
    assert np.all(mtf.mtf_radial(az, w) == pytest.approx(1.0))


def test_radial_windows_of_an_offset_cosine():
    """a + b cos(2 pi r / w) in every window of w rings: modulation b / a."""
    nr, w, a, b = 48, 8, 0.05, 0.02
    prof = a + b * np.cos(2 * math.pi * np.arange(nr) / w)
    vol = np.broadcast_to(prof[None, None, :], (2, 5, nr)).copy()
    np.testing.assert_allclose(mtf.mtf_radial(vol, w), b / a, rtol=1e-13)


def test_windows_match_loops():
    rng = np.random.default_rng(4500)
    vol = rng.uniform(0.0, 1.0, size=(6, 7, 20))
    s = 0.5 * (vol[2] + vol[3])
    for w in (1, 3, 5, 20):
        got = mtf.mtf_radial(vol, w)
        assert got.size == 20 // w
        for k in range(20 // w):
            hi = max(s[t, r] for t in range(7) for r in range(k * w, (k + 1) * w))
            lo = min(s[t, r] for t in range(7) for r in range(k * w, (k + 1) * w))
            assert got[k] == pytest.approx((hi - lo) / (hi + lo), rel=1e-15)
    az = mtf.mtf_azimuthal(vol)
    for r in range(20):
        hi, lo = max(s[:, r]), min(s[:, r])
        assert az[r] == pytest.approx((hi - lo) / (hi + lo), rel=1e-15)


def test_interleaved_order_is_a_permutation_with_a_coprime_step():
    for n in (1, 2, 3, 67, 120, 4096):
        o = I.interleaved_order(n)
        assert sorted(o.tolist()) == list(range(n))
        if n > 2:
            step = int(o[1])
            assert math.gcd(step, n) == 1 and abs(step - 0.381966 * n) <= n / 10 + 1
