"""Plain reference of the paper's own projector pair (Sec. 2.2), used as a
comparison for the exact, matched pair.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.
Written from the paper's description with numpy, in FP64:

  * forward projection, pixel driven: each ray (source -> pixel centre) is
    sampled at equal steps in Cartesian space, at distances
    d_k = (k + 1/2) step from the source while d_k < |pixel - source|; each
    sample inside the grid support (r_min <= r < r_max, h_min <= h < h_max)
    goes through the cylindrical transform (Eq. 2) and adds step * mu there:
      - nearest: mu of the cell holding the sample, so t_jl = step x (number
        of samples in cell l), the paper's intrinsic weights;
      - linear: mu interpolated on the cylindrical grid, trilinearly in
        (r, theta, h) between cell centres, theta periodic, r and h clamped
        to the first and last centres (the paper names interpolation, not
        its kind);
    the row sum of either is step x (samples in the support);
  * back-projection, voxel driven: each cell centre is projected into the
    view and the image is read there by bilinear interpolation between pixel
    centres (pixels off the detector read nothing); the same weights summed
    are the cell's column normalisation.  This is not the transpose of the
    forward projection;
  * SART (Eq. 7) with this pair: per view, rho = wp (p - q) / L over the
    sampled row sums L, c = voxel back-projection of rho, n = the
    normalisation, mu += lam w c / n where n > 0.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ref


def _grid_steps(g):
    return (g.r_max - g.r_min) / g.n_r, 2 * math.pi / g.n_theta, (g.h_max - g.h_min) / g.n_h


def _samples(a, e, step):
    """Sample points (n, 3) of the segment a -> e at distances (k + 1/2) step."""
    d = e - a
    length = float(np.linalg.norm(d))
    k = np.arange(int(math.ceil(length / step - 0.5)))
    dist = (k + 0.5) * step
    dist = dist[dist < length]
    return a[None, :] + (dist / length)[:, None] * d[None, :]


def _cyl(g, x):
    r = np.hypot(x[:, 0], x[:, 1])
    th = np.mod(np.arctan2(x[:, 1], x[:, 0]) - g.theta0, 2 * math.pi)
    return r, th, x[:, 2]


def _inside(g, r, h):
    return (r >= g.r_min) & (r < g.r_max) & (h >= g.h_min) & (h < g.h_max)


def _value(g, vol, r, th, h, mode):
    dr, dt, dh = _grid_steps(g)
    if mode == "nearest":
        ir = np.clip(np.floor((r - g.r_min) / dr).astype(int), 0, g.n_r - 1)
        ih = np.clip(np.floor((h - g.h_min) / dh).astype(int), 0, g.n_h - 1)
        it = np.clip(np.floor(th / dt).astype(int), 0, g.n_theta - 1)
        return vol[ih, it, ir]
    fr = (r - g.r_min) / dr - 0.5
    fh = (h - g.h_min) / dh - 0.5
    ft = th / dt - 0.5
    out = np.zeros_like(r)
    r0, h0, t0 = np.floor(fr).astype(int), np.floor(fh).astype(int), np.floor(ft).astype(int)
    wr, wh, wt = fr - r0, fh - h0, ft - t0
    for dh_ in (0, 1):
        ih = np.clip(h0 + dh_, 0, g.n_h - 1)
        whh = wh if dh_ else 1 - wh
        for dt_ in (0, 1):
            it = np.mod(t0 + dt_, g.n_theta)
            wtt = wt if dt_ else 1 - wt
            for dr_ in (0, 1):
                ir = np.clip(r0 + dr_, 0, g.n_r - 1)
                wrr = wr if dr_ else 1 - wr
                out += whh * wtt * wrr * vol[ih, it, ir]
    return out


def sampled_fp(scan, vol, step, mode="nearest", vb=0, ve=None):
    """(views, rows, cols) sampled projections q and row sums L."""
    o = ref.Oracle(scan)
    g = scan.grid
    vol = np.asarray(vol, dtype=np.float64).reshape(g.shape)
    ve = scan.n_views if ve is None else ve
    q = np.zeros((ve - vb, scan.det_rows, scan.det_cols))
    L = np.zeros_like(q)
    for k in range(vb, ve):
        for v in range(scan.det_rows):
            for u in range(scan.det_cols):
                a, e = o.ray_ends(k, v, u)
                x = _samples(a, e, step)
                r, th, h = _cyl(g, x)
                m = _inside(g, r, h)
                if m.any():
                    q[k - vb, v, u] = step * _value(g, vol, r[m], th[m], h[m], mode).sum()
                    L[k - vb, v, u] = step * m.sum()
    return q, L


def _object_views(scan):
    """Per view: source a, detector origin (pixel (0, 0) centre) P0 and steps
    U, V in the object frame (points X' = R X + T, directions R X)."""
    R, T = np.asarray(scan.R, float), np.asarray(scan.T, float)
    out = []
    for w in np.asarray(scan.views, float):
        S, D, U, V = w[0:3], w[3:6], w[6:9], w[9:12]
        P0 = D - 0.5 * (scan.det_cols - 1) * U - 0.5 * (scan.det_rows - 1) * V
        out.append((R @ S + T, R @ P0 + T, R @ U, R @ V))
    return out


def cell_centres(g):
    dr, dt, dh = _grid_steps(g)
    ih, it, ir = np.meshgrid(np.arange(g.n_h), np.arange(g.n_theta), np.arange(g.n_r), indexing="ij")
    r = g.r_min + (ir + 0.5) * dr
    th = g.theta0 + (it + 0.5) * dt
    h = g.h_min + (ih + 0.5) * dh
    return np.stack([r * np.cos(th), r * np.sin(th), h], axis=-1).reshape(-1, 3)


def project_points(view, x):
    """(u, v, in_front) detector coordinates (pixel indices) of points x."""
    a, P0, U, V = view
    M = np.column_stack([P0 - a, U, V])
    w = np.linalg.solve(M, (x - a).T)
    lam = w[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        return w[1] / lam, w[2] / lam, lam > 0


def voxel_bp(scan, y, vb=0, ve=None):
    """Voxel-driven back-projection of images y (ve - vb, rows, cols): per
    cell, the bilinear reading of each view at the cell centre's projection,
    summed over views; and the summed bilinear weights."""
    g = scan.grid
    ve = scan.n_views if ve is None else ve
    y = np.asarray(y, dtype=np.float64).reshape(ve - vb, scan.det_rows, scan.det_cols)
    x = cell_centres(g)
    views = _object_views(scan)
    c = np.zeros(len(x))
    n = np.zeros(len(x))
    H, W = scan.det_rows, scan.det_cols
    for k in range(vb, ve):
        u, v, front = project_points(views[k], x)
        u0, v0 = np.floor(u), np.floor(v)
        fu, fv = u - u0, v - v0
        for du in (0, 1):
            for dv in (0, 1):
                uu, vv = u0 + du, v0 + dv
                w = (fu if du else 1 - fu) * (fv if dv else 1 - fv)
                ok = front & (uu >= 0) & (uu < W) & (vv >= 0) & (vv < H)
                iu, iv = uu[ok].astype(int), vv[ok].astype(int)
                c[ok] += w[ok] * y[k - vb, iv, iu]
                n[ok] += w[ok]
    return c.reshape(g.shape), n.reshape(g.shape)


def sampled_sart(scan, proj, vol0, n_iter, step, mode="nearest", lam=0.5, proj_weights=None, vox_weights=None):
    """SART (Eq. 7, one view per update, views in order) with the paper's
    sampled forward projection and voxel-driven back-projection."""
    g = scan.grid
    mu = np.asarray(vol0, dtype=np.float64).reshape(g.shape).copy()
    p = np.asarray(proj, dtype=np.float64)
    w = np.ones(g.shape) if vox_weights is None else np.asarray(vox_weights, float).reshape(g.shape)
    for _ in range(n_iter):
        for k in range(scan.n_views):
            q, L = sampled_fp(scan, mu, step, mode, k, k + 1)
            res = p[k] - q[0]
            if proj_weights is not None:
                res = res * np.asarray(proj_weights, float)[k]
            rho = np.where(L[0] > 0, res / np.where(L[0] > 0, L[0], 1.0), 0.0)
            c, n = voxel_bp(scan, rho[None], k, k + 1)
            mu = mu + np.where(n > 0, lam * w * c / np.where(n > 0, n, 1.0), 0.0)
    return mu
