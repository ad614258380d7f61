"""Plain reference of the projection-based pose estimation (Sec. 2.1).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.
Written from the paper's description, step by step, with numpy and scipy:

  1. segmentation: pixels whose line integral exceeds a threshold, dilated by a
     (2k+1) x (2k+1) square (the paper's threshold and dilation);
  2. the four corner pixels of the segment and their pairwise centres, taken as
     two points of the projected symmetry axis per view (axis tracking);
  3. point tracking, Eq. 3-4: the 3-D point whose projections are nearest, in
     the least-squares sense, to the tracked detector points of all views,
     solved with scipy's Levenberg-Marquardt;
  4. the pose (Eq. 1) from the two tracked axis points, their heights on the
     object axis and the internal rotation angle.

Corner rule (the paper names the corners, not how ties are broken): with u the
column and v the row index, top-left minimises u + v, top-right maximises
u - v (ties: smallest v), bottom-left minimises u - v, bottom-right maximises
u + v (ties: largest v).  Top point = centre of the two top corners, bottom
point = centre of the two bottom corners.
"""
from __future__ import annotations

import math

import numpy as np


def segment(proj, threshold, k):
    """Boolean mask of one projection: value > threshold, dilated by a square of
    half-width k (every pixel within k rows and k columns of a seed pixel)."""
    seed = np.asarray(proj) > threshold
    out = seed.copy()
    H, W = seed.shape
    for dv in range(-k, k + 1):
        for du in range(-k, k + 1):
            src = seed[max(0, -dv):H - max(0, dv), max(0, -du):W - max(0, du)]
            out[max(0, dv):H - max(0, -dv), max(0, du):W - max(0, -du)] |= src
    return out


def corners(mask):
    """The four corner pixels [(u, v)] x 4 (TL, TR, BL, BR) of a mask, or None
    if it is empty."""
    v, u = np.nonzero(mask)
    if u.size == 0:
        return None
    out = []
    for key, ties_up in ((u + v, True), (-(u - v), True), (u - v, False), (-(u + v), False)):
        best = key.min()
        sel = np.nonzero(key == best)[0]
        j = sel[np.argmin(v[sel])] if ties_up else sel[np.argmax(v[sel])]
        out.append((int(u[j]), int(v[j])))
    return out


def axis_points(projs, threshold, k):
    """Per view: (top (u, v), bottom (u, v), corners) or None for an empty mask."""
    res = []
    for p in projs:
        c = corners(segment(p, threshold, k))
        if c is None:
            res.append(None)
            continue
        top = ((c[0][0] + c[1][0]) / 2.0, (c[0][1] + c[1][1]) / 2.0)
        bottom = ((c[2][0] + c[3][0]) / 2.0, (c[2][1] + c[3][1]) / 2.0)
        res.append((top, bottom, c))
    return res


def _view_matrix(view, rows, cols):
    """S and M with X - S = M (lam, lam u, lam v): pixel (u, v) at
    D + (u - (W-1)/2) U + (v - (H-1)/2) V."""
    S, D, U, V = view[0:3], view[3:6], view[6:9], view[9:12]
    d0 = D - S - 0.5 * (cols - 1) * U - 0.5 * (rows - 1) * V
    return S, np.column_stack([d0, U, V])


def project(views, rows, cols, X):
    """(n_views, 2) detector coordinates (u, v) of the stage-frame point X."""
    out = np.zeros((len(views), 2))
    for i, vw in enumerate(views):
        S, M = _view_matrix(np.asarray(vw, dtype=np.float64), rows, cols)
        w = np.linalg.solve(M, np.asarray(X, dtype=np.float64) - S)
        out[i] = (w[1] / w[0], w[2] / w[0])
    return out


def track_point(views, rows, cols, uv, valid=None, x0=None):
    """Eq. 4: argmin_X sum_i |uv_i - V_i(X)|^2 over the valid views
    (scipy Levenberg-Marquardt from x0, default the stage origin)."""
    from scipy.optimize import least_squares
    uv = np.asarray(uv, dtype=np.float64)
    keep = np.ones(len(views), bool) if valid is None else np.asarray(valid, bool)
    vs = [np.asarray(v, dtype=np.float64) for v, k in zip(views, keep) if k]
    target = uv[keep]

    def resid(X):
        return (project(vs, rows, cols, X) - target).ravel()

    sol = least_squares(resid, np.zeros(3) if x0 is None else np.asarray(x0, float), method="lm",
                        xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
    rms = float(np.sqrt(np.mean(sol.fun ** 2)))
    return sol.x, rms


def pose_from_axis(top, bottom, h_top, h_bottom, alpha):
    """(R, T) of Eq. 1 (X' = R X + T, R = Rz(alpha) Rx(beta) Rz(gamma)) from two
    stage-frame points of the object axis at heights h_top > h_bottom, and the
    internal rotation alpha.  The object axis in the stage frame is
    R^T z = (sin b sin g, sin b cos g, cos b)."""
    top = np.asarray(top, float)
    bottom = np.asarray(bottom, float)
    d = (top - bottom) / np.linalg.norm(top - bottom)
    beta = float(np.arccos(np.clip(d[2], -1.0, 1.0)))
    gamma = float(np.arctan2(d[0], d[1])) if np.hypot(d[0], d[1]) > 0 else 0.0
    ca, sa = np.cos(alpha), np.sin(alpha)
    cb, sb = np.cos(beta), np.sin(beta)
    cg, sg = np.cos(gamma), np.sin(gamma)
    Rz_a = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1.0]])
    Rx_b = np.array([[1.0, 0, 0], [0, cb, -sb], [0, sb, cb]])
    Rz_g = np.array([[cg, -sg, 0], [sg, cg, 0], [0, 0, 1.0]])
    R = Rz_a @ Rx_b @ Rz_g
    centre = 0.5 * (top + bottom) - 0.5 * (h_top + h_bottom) * d
    return R, -R @ centre


# ---------------------------------------------------------------- azimuthal phase

def side_sums(projs, centres, row_lo, row_hi):
    """Per view k: (grey-value sum left of the detector position centres[k],
    sum right of it) over rows [row_lo[k], row_hi[k]] (inclusive, clipped): the
    grey values beside the projected axis.  Pixel u spans [u - 1/2, u + 1/2]
    and is split at the centre in proportion, so an object symmetric about the
    axis gives equal sums wherever the axis falls."""
    out = np.zeros((len(projs), 2))
    for k, p in enumerate(projs):
        H, W = p.shape
        a, b = max(0, int(row_lo[k])), min(H - 1, int(row_hi[k]))
        if a > b:
            continue
        u = np.arange(W)
        f_left = np.clip(centres[k] - (u - 0.5), 0.0, 1.0)
        col = np.asarray(p[a:b + 1], dtype=np.float64).sum(axis=0)
        out[k, 0] = (col * f_left).sum()
        out[k, 1] = (col * (1.0 - f_left)).sum()
    return out


def azimuth_phase(s, s_ref):
    """The internal rotation a maximising the circular cross-correlation
    C(t) = integral s(phi) s_ref(phi + t) dphi of two signals sampled at the N
    equally spaced view angles of a full circular trajectory (phi_k = phi_0 +
    2 pi k / N).  Shifting the view angle is rotating the object about the
    rotation axis, so the measured grey-value signal is the reference one
    advanced by the object's internal rotation (Sec. 2.1, azimuthal phase; the
    reference is projected with the same axis pose, which carries the tilt
    correction of Eq. 5).  With the discrete Fourier coefficients S_m, R_m
    (m = 1 .. floor((N-1)/2)), C(t) = sum_m 2 |S_m R_m| cos(m t - arg(S_m conj R_m));
    its maximum on a 0.1-degree grid is refined by Newton steps."""
    s = np.asarray(s, float)
    r = np.asarray(s_ref, float)
    N = s.size
    S = np.fft.rfft(s)
    R = np.fft.rfft(r)
    M = (N - 1) // 2
    m = np.arange(1, M + 1)
    X = S[1:M + 1] * np.conj(R[1:M + 1])
    amp, th = 2 * np.abs(X), np.angle(X)
    taus = np.arange(3600) * (2 * np.pi / 3600)
    C = (amp[None, :] * np.cos(np.outer(taus, m) - th[None, :])).sum(axis=1)
    t = taus[int(np.argmax(C))]
    for _ in range(8):
        d1 = -(amp * m * np.sin(m * t - th)).sum()
        d2 = -(amp * m * m * np.cos(m * t - th)).sum()
        if d2 >= 0:
            break
        t -= d1 / d2
    return float(np.mod(t, 2 * np.pi))


def gamma_eq5(phi_p, phi_g, a1, a2):
    """Sec. 2.1, Eq. 5: the last Euler angle from the perceived phase phi_p,
    the geometric angle phi_g and the first two Euler angles a1, a2:
    phi_p - phi_g - arctan(tan(a1) / cos(a2)), the arctangent continued
    through a1 = +-pi/2 (atan2(sin a1, cos a1 cos a2)), wrapped to [0, 2 pi)."""
    corr = math.atan2(math.sin(a1), math.cos(a1) * math.cos(a2))
    g = phi_p - phi_g - corr
    return g - 2.0 * math.pi * math.floor(g / (2.0 * math.pi))
