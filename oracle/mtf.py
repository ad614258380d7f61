"""Plain reference of the directional MTF measurement (Sec. 2.3, Eq. 8).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.
Written from the paper's description with numpy, in FP64:

  * the central slice: the middle h-slice of the volume, or the mean of the
    two middle slices when N_h is even (the paper does not say which slice
    an even N_h uses);
  * the modulation of a set of values, Eq. 8:
        m = (mu_max - mu_min) / (mu_max + mu_min)     (0 when both are 0);
  * the azimuthal MTF at each radius: the modulation over theta of one ring
    of the central slice;
  * the radial MTF's radial dependence: windows of one phantom period (w
    rings) slid by their own width, each the modulation over all cells of
    the central slice in those rings;
  * the whole-slice modulation.

Volumes are (N_h, N_theta, N_r), r fastest.
"""
from __future__ import annotations

import numpy as np


def central_slice(vol):
    """(N_theta, N_r) central h-slice in FP64: the middle slice, or the mean of
    the two middle ones for even N_h."""
    v = np.asarray(vol, dtype=np.float64)
    nh = v.shape[0]
    if nh % 2:
        return v[nh // 2].copy()
    return 0.5 * (v[nh // 2 - 1] + v[nh // 2])


def modulation(values):
    """Eq. 8 over a set of values."""
    x = np.asarray(values, dtype=np.float64)
    hi, lo = float(x.max()), float(x.min())
    return 0.0 if hi + lo == 0.0 else (hi - lo) / (hi + lo)


def mtf_azimuthal(vol):
    """(N_r,) modulation over theta of each ring of the central slice."""
    s = central_slice(vol)
    return np.array([modulation(s[:, r]) for r in range(s.shape[1])])


def mtf_radial(vol, width):
    """(N_r // width,) modulation over the cells of each window of `width`
    rings of the central slice, windows [k w, (k + 1) w)."""
    s = central_slice(vol)
    n = s.shape[1] // width
    return np.array([modulation(s[:, k * width:(k + 1) * width]) for k in range(n)])


def mtf_slice(vol):
    """Modulation over the whole central slice."""
    return modulation(central_slice(vol))
