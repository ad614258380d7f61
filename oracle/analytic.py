"""Closed-form chord lengths that pin the oracle (TEST INFRASTRUCTURE ONLY).

Every ring-sector box [h0,h1) x [th0,th1) x [r0,r1) on the cylindrical grid
(Sec. 2, Eq. 2) is slab ∩ wedge ∩ disc(r1) minus the same set inside disc(r0).
For a wedge no wider than pi, slab, wedge and disc are all convex, so a ray
meets each of slab ∩ wedge ∩ disc(r) in one parameter interval and

    chord = |d| * ( |I_slab ∩ I_wedge ∩ I_disc(r1)| - |I_slab ∩ I_wedge ∩ I_disc(r0)| )

with the slab interval linear in t, the wedge interval from two half-plane
inequalities and the disc interval from the shell quadric.  This is interval
algebra per (ray, box): it shares nothing with the oracle's sort-and-classify
method, so agreement between the two pins the oracle's system matrix (Eq. 6).

All functions are vectorised over rays: a, e are (n, 3) arrays of object-frame
source and pixel-centre points, t in [0, 1] along a -> e.
"""
from __future__ import annotations

import math

import numpy as np


def _iv_and(lo1, hi1, lo2, hi2):
    return np.maximum(lo1, lo2), np.minimum(hi1, hi2)


def _iv_len(lo, hi):
    return np.maximum(hi - lo, 0.0)


def segment_interval(n):
    return np.zeros(n), np.ones(n)


def slab_interval(a, d, z0, z1):
    """t-interval with z0 <= a_z + t d_z <= z1."""
    az, dz = a[:, 2], d[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (z0 - az) / dz
        t1 = (z1 - az) / dz
    lo = np.minimum(t0, t1)
    hi = np.maximum(t0, t1)
    par = dz == 0.0
    inside = (az >= z0) & (az < z1)
    lo = np.where(par, np.where(inside, -np.inf, np.inf), lo)
    hi = np.where(par, np.where(inside, np.inf, -np.inf), hi)
    return lo, hi


def disc_interval(a, d, rho):
    """t-interval with (a_x + t d_x)^2 + (a_y + t d_y)^2 <= rho^2."""
    n = a.shape[0]
    if rho <= 0.0:
        return np.full(n, np.inf), np.full(n, -np.inf)
    A = d[:, 0] ** 2 + d[:, 1] ** 2
    B = a[:, 0] * d[:, 0] + a[:, 1] * d[:, 1]
    Cc = a[:, 0] ** 2 + a[:, 1] ** 2 - rho * rho
    disc = B * B - A * Cc
    with np.errstate(divide="ignore", invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0.0))
        q = -(B + np.copysign(sq, B))
        r1 = q / A
        r2 = Cc / q
    lo = np.minimum(r1, r2)
    hi = np.maximum(r1, r2)
    ok = (A > 0) & (disc > 0)
    # a ray parallel to the axis is inside the disc for all t or for none
    par = A == 0.0
    par_in = Cc < 0.0
    lo = np.where(ok, lo, np.where(par & par_in, -np.inf, np.inf))
    hi = np.where(ok, hi, np.where(par & par_in, np.inf, -np.inf))
    return lo, hi


def halfplane_interval(a, d, theta, sign):
    """t-interval with sign * n(theta).(a + t d)_xy >= 0, n = (-sin, cos)."""
    nx, ny = -math.sin(theta) * sign, math.cos(theta) * sign
    na = nx * a[:, 0] + ny * a[:, 1]
    nd = nx * d[:, 0] + ny * d[:, 1]
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -na / nd
    lo = np.where(nd > 0, t, -np.inf)
    hi = np.where(nd < 0, t, np.inf)
    zero = nd == 0
    lo = np.where(zero, np.where(na >= 0, -np.inf, np.inf), lo)
    hi = np.where(zero, np.where(na >= 0, np.inf, -np.inf), hi)
    return lo, hi


def wedge_interval(a, d, th0, th1):
    """t-interval of the convex wedge th0 <= theta <= th1 (th1 - th0 <= pi)."""
    assert th1 - th0 <= math.pi + 1e-12
    lo1, hi1 = halfplane_interval(a, d, th0, +1.0)
    lo2, hi2 = halfplane_interval(a, d, th1, -1.0)
    return _iv_and(lo1, hi1, lo2, hi2)


def _theta_pieces(grid, it0, it1):
    """Split the sector range [it0, it1) (may exceed N_theta: wraps) into
    angle ranges no wider than pi; None means the full circle."""
    nt = grid.n_theta
    if it1 - it0 >= nt:
        return None
    dth = 2 * math.pi / nt
    th0 = grid.theta0 + it0 * dth
    th1 = grid.theta0 + it1 * dth
    pieces = []
    while th1 - th0 > math.pi:
        pieces.append((th0, th0 + math.pi))
        th0 += math.pi
    pieces.append((th0, th1))
    return pieces


def box_chord(grid, a, e, ih0, ih1, it0, it1, ir0, ir1):
    """Length of each ray a->e inside the ring-sector box of the grid."""
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    e = np.atleast_2d(np.asarray(e, dtype=np.float64))
    d = e - a
    n = a.shape[0]
    dh = (grid.h_max - grid.h_min) / grid.n_h
    dr = (grid.r_max - grid.r_min) / grid.n_r
    z0, z1 = grid.h_min + ih0 * dh, grid.h_min + ih1 * dh
    r0, r1 = grid.r_min + ir0 * dr, grid.r_min + ir1 * dr
    slo, shi = _iv_and(*segment_interval(n), *slab_interval(a, d, z0, z1))
    pieces = _theta_pieces(grid, it0, it1)
    if pieces is None:
        wl = [(np.full(n, -np.inf), np.full(n, np.inf))]
    else:
        wl = [wedge_interval(a, d, p0, p1) for (p0, p1) in pieces]
    olo, ohi = disc_interval(a, d, r1)
    ilo, ihi = disc_interval(a, d, r0)
    total = np.zeros(n)
    for (wlo, whi) in wl:
        lo, hi = _iv_and(slo, shi, wlo, whi)
        total += _iv_len(*_iv_and(lo, hi, olo, ohi)) - _iv_len(*_iv_and(lo, hi, ilo, ihi))
    return total * np.linalg.norm(d, axis=1)


def support_chord(grid, a, e):
    """Row sum L_j: the ray's length inside the whole grid support."""
    return box_chord(grid, a, e, 0, grid.n_h, 0, grid.n_theta, 0, grid.n_r)


def dense_matrix(grid, a, e):
    """Brute force: A[j, l] for every ray j and every cell l by per-cell
    interval algebra (tiny grids only)."""
    a = np.atleast_2d(a)
    e = np.atleast_2d(e)
    nh, nt, nr = grid.n_h, grid.n_theta, grid.n_r
    A = np.zeros((a.shape[0], nh * nt * nr))
    for ih in range(nh):
        for it in range(nt):
            for ir in range(nr):
                l = (ih * nt + it) * nr + ir
                A[:, l] = box_chord(grid, a, e, ih, ih + 1, it, it + 1, ir, ir + 1)
    return A


def boxes_projection(grid, a, e, boxes):
    """sum_b coef_b * chord(box_b) for boxes (coef, ih0, ih1, it0, it1, ir0, ir1)."""
    a = np.atleast_2d(a)
    out = np.zeros(a.shape[0])
    for (coef, ih0, ih1, it0, it1, ir0, ir1) in boxes:
        out += coef * box_chord(grid, a, e, ih0, ih1, it0, it1, ir0, ir1)
    return out


def _box_and(b1, b2, nt):
    """Intersection of two index boxes (theta ranges given with it0 in [0, nt));
    returns a list (theta wrap can split it in two)."""
    (h0, h1, t0, t1, r0, r1) = b1
    (H0, H1, T0, T1, R0, R1) = b2
    hh0, hh1 = max(h0, H0), min(h1, H1)
    rr0, rr1 = max(r0, R0), min(r1, R1)
    if hh0 >= hh1 or rr0 >= rr1:
        return []
    out = []
    for shift in (-nt, 0, nt):
        a0, a1 = max(t0, T0 + shift), min(t1, T1 + shift)
        if a0 < a1:
            out.append((hh0, hh1, a0, a1, rr0, rr1))
    return out


def painted_boxes(grid, layers):
    """Signed boxes whose sum equals a volume painted layer by layer.

    layers: [(mu, ih0, ih1, it0, it1, ir0, ir1)], later layers overwrite
    earlier ones (painter's order).  Painting box B with mu over f gives
    f - f*1_B + mu*1_B, applied to the box list."""
    nt = grid.n_theta
    boxes = []  # (coef, box)
    for (mu, ih0, ih1, it0, it1, ir0, ir1) in layers:
        B = (ih0, ih1, it0, it1, ir0, ir1)
        new = list(boxes)
        for (c, b) in boxes:
            for x in _box_and(b, B, nt):
                new.append((-c, x))
        new.append((mu, B))
        boxes = [(c, b) for (c, b) in new if c != 0.0]
    return [(c,) + tuple(b) for (c, b) in boxes]


def paint(grid, layers):
    """The painted volume itself (for comparison with the box sum)."""
    vol = np.zeros(grid.shape)
    nt = grid.n_theta
    for (mu, ih0, ih1, it0, it1, ir0, ir1) in layers:
        vol[ih0:ih1, np.arange(it0, it1) % nt, ir0:ir1] = mu
    return vol
