"""Pins of the oracle's ordered-subset SART (Eq. 7 with an ordered subset of
several projections, up to SIRT) against facts that do not come from it:

* one update per group written out with the brute-force system matrix of
  oracle/analytic.py (per-(ray, cell) interval algebra, no shared code), for
  ragged groups, a permuted view order, pixel and voxel weights and a posed
  object,
* the single-voxel closed form mu_K = mu* + (1 - lam)^K (mu_0 - mu*) after K
  group updates on consistent data,
* subset 1 = the one-projection sweep, bit for bit,
* SIRT (all views in one group) never increases the residual weighted by the
  inverse row sums when lam <= 1 (the normalised matrix has norm <= 1),
* resume at a group boundary.
"""
import numpy as np
import pytest

from oracle import analytic
from paper_2005_11976_amd import inputs as I


def _rays(o, scan, k):
    a, e = [], []
    for v in range(scan.det_rows):
        for u in range(scan.det_cols):
            aa, ee = o.ray_ends(k, v, u)
            a.append(aa)
            e.append(ee)
    return np.array(a), np.array(e)


def _tiny(posed):
    grid = I.Grid(3, 8, 3, 0.5, 6.0, -3.0, 3.0, 0.2)
    views = I.circular_views(5, 40.0, 80.0, 1.1, 0.9, phi0=0.17)
    R, T = I.pose_from(0.4, 0.3, 1.1, [0.7, -0.4, 0.5]) if posed else I.identity_pose()
    return I.Scan(grid, np.asarray(views, dtype=np.float64), 8, 6, R, T)


def _explicit_os(mats, p, mu0, n_iter, m, lam, order, pw=None, vw=None):
    """Eq. 7 per group of m consecutive positions of `order`, with the
    explicit per-view matrices A_k (rays x cells)."""
    mu = mu0.ravel().astype(np.float64).copy()
    N = len(mats)
    w = np.ones_like(mu) if vw is None else vw.ravel()
    for _ in range(n_iter):
        for g0 in range(0, N, m):
            group = order[g0:g0 + m]
            c = np.zeros_like(mu)
            n = np.zeros_like(mu)
            rhos = []
            for k in group:  # residuals of the whole group from the same mu
                A = mats[k]
                L = A.sum(axis=1)
                res = p[k].ravel() - A @ mu
                if pw is not None:
                    res = res * pw[k].ravel()
                rhos.append(np.where(L > 0, res / np.where(L > 0, L, 1.0), 0.0))
            for k, rho in zip(group, rhos):
                c += mats[k].T @ rho
                n += mats[k].sum(axis=0)
            mu = mu + np.where(n > 0, lam * w * c / np.where(n > 0, n, 1.0), 0.0)
    return mu


@pytest.mark.parametrize("posed", [False, True])
@pytest.mark.parametrize("m", [2, 3, 5, 9])
def test_os_update_matches_explicit_matrix(oracle_mod, posed, m):
    scan = _tiny(posed)
    o = oracle_mod.Oracle(scan)
    mats = [analytic.dense_matrix(scan.grid, *_rays(o, scan, k)) for k in range(scan.n_views)]
    rng = np.random.default_rng(4400 + m)
    truth = rng.uniform(0.0, 0.05, size=scan.grid.shape)
    p = np.stack([(A @ truth.ravel()).reshape(scan.det_rows, scan.det_cols) for A in mats])
    p = p + rng.normal(0.0, 0.01, size=p.shape)  # inconsistent data: every view moves mu
    mu0 = rng.uniform(0.0, 0.05, size=scan.grid.shape)
    pw = rng.uniform(0.5, 1.0, size=p.shape)
    vw = rng.uniform(0.25, 1.0, size=scan.grid.shape)
    order = np.array([3, 0, 4, 1, 2], dtype=np.int32)
    got, _ = o.sart(p, mu0, 2, 0.7, proj_weights=pw, vox_weights=vw, view_order=order, subset=m)
    want = _explicit_os(mats, p, mu0, 2, min(m, scan.n_views), 0.7, list(order), pw, vw)
    assert np.abs(want - mu0.ravel()).max() > 1e-3
    np.testing.assert_allclose(got.ravel(), want, rtol=1e-11, atol=1e-14)


def test_os_single_voxel_closed_form(oracle_mod):
    grid = I.Grid(1, 1, 1, 0.0, 5.0, -5.0, 5.0)
    views = I.circular_views(5, 50.0, 100.0, 0.5, 0.5, phi0=0.3)
    scan = I.Scan(grid, np.asarray(views, dtype=np.float64), 3, 3, *I.identity_pose())
    o = oracle_mod.Oracle(scan)
    mu_star, mu0, lam = 0.04, 0.01, 0.6
    p = o.fp(np.full(grid.shape, mu_star))
    assert (o.fp(np.ones(grid.shape)) > 0).all()  # every ray meets the voxel
    for m, groups_per_iter in ((1, 5), (2, 3), (5, 1)):
        for n_iter in (1, 2):
            mu, _ = o.sart(p, np.full(grid.shape, mu0), n_iter, lam, subset=m)
            K = n_iter * groups_per_iter
            assert mu.ravel()[0] == pytest.approx(mu_star + (1 - lam) ** K * (mu0 - mu_star), rel=1e-12)


def test_os_subset_one_is_the_single_view_sweep(oracle_mod):
    scan = I.scaled_single(n_h=8, n_theta=24, n_r=6, n_views=10, det=20, posed_seed=2005)
    ph = I.industrial_phantom(scan.grid, 77, n_annuli=4, n_incl=3)
    o = oracle_mod.Oracle(scan)
    p = o.fp(ph.truth)
    a, ra = o.sart(p, ph.prior, 2, 0.5, vox_weights=ph.weights, nthreads=4)
    b, rb = o.sart(p, ph.prior, 2, 0.5, vox_weights=ph.weights, nthreads=4, subset=1)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_sirt_weighted_residual_does_not_increase(oracle_mod):
    scan = I.scaled_single(n_h=8, n_theta=24, n_r=6, n_views=10, det=20)
    ph = I.industrial_phantom(scan.grid, 78, n_annuli=4, n_incl=3)
    o = oracle_mod.Oracle(scan)
    p = o.fp(ph.truth)
    L = o.row_sums()
    inv = np.where(L > 0, 1.0 / np.where(L > 0, L, 1.0), 0.0)
    mu = np.zeros(scan.grid.shape)
    prev = float((inv * (p - o.fp(mu)) ** 2).sum())
    for _ in range(4):
        mu, _ = o.sart(p, mu, 1, 1.0, subset=scan.n_views, nthreads=4)
        cur = float((inv * (p - o.fp(mu)) ** 2).sum())
        assert cur <= prev * (1 + 1e-12)
        prev = cur
    assert prev < 0.5 * float((inv * p ** 2).sum())


def test_os_resume_at_group_boundary(oracle_mod):
    scan = I.scaled_single(n_h=8, n_theta=24, n_r=6, n_views=10, det=20)
    ph = I.industrial_phantom(scan.grid, 79, n_annuli=4, n_incl=3)
    o = oracle_mod.Oracle(scan)
    p = o.fp(ph.truth)
    full, _ = o.sart(p, ph.prior, 2, 0.5, subset=4, nthreads=4)
    first = I.Scan(scan.grid, scan.views[:4], scan.det_rows, scan.det_cols, scan.R, scan.T)
    g1, _ = oracle_mod.Oracle(first).sart(p[:4], ph.prior, 1, 0.5, subset=4, nthreads=4)
    rest, _ = o.sart(p, g1, 2, 0.5, subset=4, start_view=4, nthreads=4)
    assert np.array_equal(full, rest)
