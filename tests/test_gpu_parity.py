"""GPU parity of the HIP projectors and SART against the FP64 oracle.

Every call goes through the C ABI (libcyl.so via the ctypes binding).  Bars:
  * cyl_fp and cyl_bp: relative L2 <= 1e-5 against the oracle, on every grid,
    and the largest error of one ray sum or one cell at most 2e-4 of the
    largest value (a cell that a ray meets within FP32 rounding of its face
    may take or lose that rounding's length, so single cells are held to the
    array's scale, not their own);
  * adjoint <Ax, y> vs <x, A^T y> (FP64 dot products on the host): <= 1e-6;
  * row sums (closed form, FP64 on the device): relative L2 <= 1e-7;
  * SART iterates: relative L2 against the oracle's iterates at most about
    ten times what the test measured when it was written (the GPU results
    are deterministic, bit for bit, so the measured value does not drift);
  * invariants exact (bitwise): fixed point, zero weights, resume, determinism.
"""
import math

import numpy as np
import pytest

from oracle import ref
from paper_2005_11976_amd import inputs as I
from tests.gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

FP_TOL = 1e-5
BP_TOL = 1e-5
ADJ_TOL = 1e-6
ABS_TOL = 2e-4  # max |got - ref| / max |ref|


def abs_rel(got, ref):
    """Largest absolute error relative to the largest reference value."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_11976_amd import cyl
    cyl.lib()
    return torch


def _geom(scan):
    from paper_2005_11976_amd import cyl
    return cyl.Geometry(scan, 0)


def _edge_scans():
    out = []
    views = I.circular_views(5, 40.0, 80.0, 1.1, 0.9, phi0=0.17)
    R, T = I.pose_from(0.4, 0.3, 1.1, [0.7, -0.4, 0.5])
    for name, grid in [
        ("hollow", I.Grid(4, 8, 4, 1.5, 6.0, -2.0, 4.0, 0.3)),
        ("ntheta1", I.Grid(3, 1, 3, 0.0, 6.0, -3.0, 3.0)),
        ("ntheta2", I.Grid(3, 2, 2, 0.0, 6.0, -3.0, 3.0, 1.0)),
        ("ntheta3", I.Grid(2, 3, 2, 0.0, 6.0, -3.0, 3.0)),
        ("one_cell", I.Grid(1, 1, 1, 0.0, 6.0, -3.0, 3.0)),
        ("ragged_blocks", I.Grid(7, 37, 19, 0.0, 6.0, -3.0, 3.0)),
    ]:
        out.append((name, I.Scan(grid, views, 8, 6, np.eye(3), np.zeros(3))))
        out.append((name + "_posed", I.Scan(grid, views, 8, 6, R, T)))
    # odd detector: the central column's rays pass exactly through the axis
    # (theta0 keeps them off the sector-edge planes; in-plane rays are a tie
    # case checked by sums only, below)
    g = I.Grid(6, 24, 6, 0.0, 6.0, -3.0, 3.0, 0.05)
    out.append(("through_axis", I.Scan(g, I.circular_views(4, 40.0, 80.0, 0.7), 9, 11,
                                       np.eye(3), np.zeros(3))))
    # ragged 8x8 tiles and a tilted object
    R2, T2 = I.pose_from(1.0, math.radians(25.0), 0.2, [0.3, 0.1, -0.2])
    out.append(("tilted25_ragged_tiles", I.Scan(I.Grid(10, 30, 8, 0.0, 6.0, -4.0, 4.0),
                                                I.circular_views(3, 40.0, 80.0, 0.6), 21, 13, R2, T2)))
    return out


EDGE = _edge_scans()


def _fp_bp_check(torch, scan, vb, ve, seed, label, fp_tol=FP_TOL, bp_tol=BP_TOL):
    o = ref.Oracle(scan)
    G = _geom(scan)
    x = I.uniform_vector(scan.grid.n_vox, seed)
    y = I.uniform_vector(scan.n_views * scan.det_rows * scan.det_cols, seed + 1)
    say(label, "fp", scan.grid.shape, scan.proj_shape, (vb, ve))
    xg = dev(x.astype(np.float32).reshape(scan.grid.shape))
    q = host(G.fp(xg, view_begin=vb, view_end=ve))[vb:ve]
    q_ref = o.fp(x.astype(np.float32).astype(np.float64), vb, ve)
    e_fp = rel_l2(q, q_ref)
    say(label, "bp")
    yg = dev(y.astype(np.float32).reshape(scan.proj_shape))
    b = host(G.bp(yg, view_begin=vb, view_end=ve))
    y_ref = y.astype(np.float32).astype(np.float64).reshape(scan.proj_shape)[vb:ve]
    b_ref = o.bp(y_ref, vb, ve)
    e_bp = rel_l2(b, b_ref)
    lhs = float(q.ravel() @ y_ref.ravel())
    rhs = float(x.astype(np.float32).astype(np.float64) @ b.ravel())
    e_adj = abs(lhs - rhs) / abs(lhs)
    a_fp, a_bp = abs_rel(q, q_ref), abs_rel(b, b_ref)
    say(label, "fp %.2e (max abs %.2e of max) bp %.2e (max abs %.2e of max) adjoint %.2e" %
        (e_fp, a_fp, e_bp, a_bp, e_adj))
    assert e_fp <= fp_tol and a_fp <= ABS_TOL
    assert e_bp <= bp_tol and a_bp <= ABS_TOL
    assert e_adj <= ADJ_TOL
    return q, b


def test_fp_bp_tiny_all_views(torch_cuda):
    cfg = I.config_tiny()
    _fp_bp_check(torch_cuda, cfg["scan"], 0, cfg["scan"].n_views, 4001, "tiny")


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
def test_fp_bp_edge_grids(torch_cuda, case):
    name, scan = case
    _fp_bp_check(torch_cuda, scan, 0, scan.n_views, 4011, name)


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
def test_sart_edge_grids(torch_cuda, case):
    """Weighted SART from a random prior on the edge grids (one, two and three
    sectors, one cell, a hollow grid, ragged blocks, rays through the axis, a
    25 degree tilt): the super-block update on degenerate shapes against the
    oracle, 2 iterations."""
    name, scan = case
    rng = np.random.default_rng(4050)
    truth = rng.uniform(0.0, 1.0, size=scan.grid.shape)
    prior = truth * rng.uniform(0.8, 1.2, size=scan.grid.shape)
    wv = rng.uniform(0.25, 1.0, size=scan.grid.shape)
    o = ref.Oracle(scan)
    p = o.fp(truth)
    G = _geom(scan)
    pg, wg = dev(p.astype(np.float32)), dev(wv.astype(np.float32))
    vol = dev(prior.astype(np.float32))
    mu = prior.astype(np.float32).astype(np.float64)
    for it in range(2):
        say(name, "sart iteration", it)
        G.sart(pg, vol, it + 1, 0.5, vox_weights=wg, start_iter=it)
        mu, _ = o.sart(p.astype(np.float32).astype(np.float64), mu, it + 1, 0.5, vox_weights=wv.astype(np.float32),
                       start_iter=it)
        e = rel_l2(host(vol), mu)
        say(name, "sart iteration %d rel L2 %.2e" % (it, e))
        assert e <= 3e-6  # measured at most 2.7e-7


THROUGH_AXIS = [(phi0, th0, rot) for phi0 in (0.0, 0.3, 1.1) for th0 in (0.05, 0.13) for rot in (0.0, 0.7)
                if rot == 0.0 or phi0 == 0.3]


@pytest.mark.parametrize("phi0,th0,rot", THROUGH_AXIS)
def test_fp_bp_rays_through_the_axis(torch_cuda, phi0, th0, rot):
    """Odd detectors whose central column passes through the axis (to FP64
    rounding) in every view, at several scan phases, sector offsets and
    rotations about the axis: the sector such a ray leaves the axis into is
    decided at a point where its FP32 coordinates are all rounding, in the
    forward walk (ray pieces) and in the back-projection (super-blocks whose
    wedge meets the axis).  FP, BP and adjoint against the oracle."""
    g = I.Grid(6, 24, 6, 0.0, 6.0, -3.0, 3.0, th0)
    R, T = I.pose_from(0.0, 0.0, rot, [0.0, 0.0, 0.0])
    scan = I.Scan(g, I.circular_views(4, 40.0, 80.0, 0.7, phi0=phi0), 9, 11, R, T)
    _fp_bp_check(torch_cuda, scan, 0, scan.n_views, 4085, "through axis phi0 %.2f th0 %.2f rot %.1f" % (phi0, th0, rot))


def test_rays_in_sector_edge_planes_sums(torch_cuda):
    """Rays lying exactly in a sector-edge plane (and through the axis): the
    side they are given is a rounding tie, so compare what is unique: the FP
    of a theta-independent volume, and the BP summed over theta."""
    g = I.Grid(6, 24, 6, 0.0, 6.0, -3.0, 3.0)
    scan = I.Scan(g, I.circular_views(4, 40.0, 80.0, 0.7), 9, 11, np.eye(3), np.zeros(3))
    o = ref.Oracle(scan)
    G = _geom(scan)
    hr = I.uniform_vector(g.n_h * g.n_r, 21).reshape(g.n_h, 1, g.n_r)
    x = np.repeat(hr, g.n_theta, axis=1).astype(np.float32)
    say("in-plane rays fp")
    q = host(G.fp(dev(x)))
    assert rel_l2(q, o.fp(x.astype(np.float64))) <= FP_TOL
    y = I.uniform_vector(scan.n_views * scan.det_rows * scan.det_cols, 22).astype(np.float32)
    say("in-plane rays bp")
    b = host(G.bp(dev(y.reshape(scan.proj_shape))))
    b_ref = o.bp(y.astype(np.float64))
    assert rel_l2(b.sum(axis=1), b_ref.sum(axis=1)) <= BP_TOL


def test_fp_bp_view_subrange_and_accumulate(torch_cuda):
    scan = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=6, det=40, posed_seed=2005)
    G = _geom(scan)
    o = ref.Oracle(scan)
    x = I.uniform_vector(scan.grid.n_vox, 5).astype(np.float32)
    xg = dev(x.reshape(scan.grid.shape))
    say("subrange fp")
    p = torch_cuda.full(scan.proj_shape, -7.0, device="cuda")
    G.fp(xg, p, view_begin=2, view_end=4)
    ph = host(p)
    assert np.all(ph[:2] == -7.0) and np.all(ph[4:] == -7.0)
    assert rel_l2(ph[2:4], o.fp(x.astype(np.float64), 2, 4)) <= FP_TOL
    # empty range is a no-op
    G.fp(xg, p, view_begin=3, view_end=3)
    assert np.array_equal(host(p), ph)
    say("subrange bp accumulate")
    y = I.uniform_vector(scan.n_views * scan.det_rows * scan.det_cols, 6).astype(np.float32)
    yg = dev(y.reshape(scan.proj_shape))
    b = G.bp(yg, view_begin=0, view_end=3)
    G.bp(yg, b, view_begin=3, view_end=6, accumulate=True)
    ball = G.bp(yg)
    assert rel_l2(host(b), host(ball)) <= 1e-6
    assert rel_l2(host(ball), o.bp(y.astype(np.float64))) <= BP_TOL


def test_row_sums_closed_form(torch_cuda):
    from oracle import analytic
    for scan in (I.config_tiny()["scan"], EDGE[1][1], EDGE[-1][1]):
        say("row sums", scan.grid.shape)
        G = _geom(scan)
        o = ref.Oracle(scan)
        Lg = host(G.row_sums())
        Lr = o.row_sums()
        assert rel_l2(Lg, Lr) <= 1e-7
        a, e = o.ray_ends(0, 0, 0)
        assert Lg[0, 0, 0] == pytest.approx(analytic.support_chord(scan.grid, a[None], e[None])[0],
                                            rel=1e-6, abs=1e-6)


def test_single_scan_full_size_fp_sampled(torch_cuda):
    """256x720x128, 120 views: FP of the whole scan on the GPU, sampled rays
    against the oracle (unposed and posed)."""
    cfg = I.config_single()
    for posed in (False, True):
        scan = cfg["scan"]
        if posed:
            R, T, _ = I.random_pose(2002)
            scan = I.Scan(scan.grid, scan.views, scan.det_rows, scan.det_cols, R, T)
        say("single full fp posed=%s" % posed)
        G = _geom(scan)
        ph = I.industrial_phantom(scan.grid, cfg["seed"])
        x = ph.truth.astype(np.float32)
        q = host(G.fp(dev(x)))
        rng = np.random.default_rng(99)
        o = ref.Oracle(scan)
        P = scan.det_rows * scan.det_cols
        errs_num, errs_den = 0.0, 0.0
        for k in rng.choice(scan.n_views, size=6, replace=False):
            rays = rng.choice(P, size=500, replace=False)
            qr, _ = o.fp_rays(x.astype(np.float64), rays, vb=int(k))
            qg = q[int(k)].ravel()[rays]
            errs_num += float(np.sum((qg - qr) ** 2))
            errs_den += float(np.sum(qr ** 2))
        e = math.sqrt(errs_num / errs_den)
        say("single full fp posed=%s sampled rel L2 %.2e" % (posed, e))
        assert e <= FP_TOL


def test_single_scan_full_size_bp_one_view(torch_cuda):
    """256x720x128: BP of one full 512x512 view against the oracle, plus the
    adjoint identity on that view."""
    cfg = I.config_single()
    R, T, _ = I.random_pose(2002)
    scan = I.Scan(cfg["scan"].grid, cfg["scan"].views, 512, 512, R, T)
    _fp_bp_check(torch_cuda, scan, 17, 18, 4021, "single posed view 17")


def test_single_scan_full_size_bp_all_views_is_sum_of_views(torch_cuda):
    """256x720x128, 120 views: cyl_bp over all views in one call (one
    fixed-point scale per super-block for all of them) equals the sum of the
    120 one-view calls (each the one-view transpose checked against the
    oracle above), within 1e-6; and the FP of the whole scan in one call
    (one ray per lane) equals one-view calls (rays split over 4 lanes), within
    1e-6."""
    torch = torch_cuda
    cfg = I.config_single()
    scan = cfg["scan"]
    G = _geom(scan)
    y = dev(I.uniform_vector(scan.n_views * scan.det_rows * scan.det_cols, 4060).astype(np.float32)
            .reshape(scan.proj_shape))
    say("full bp all views")
    whole = host(G.bp(y))
    acc = dev(np.zeros(scan.grid.shape, np.float32))
    for k in range(scan.n_views):
        G.bp(y, acc, view_begin=k, view_end=k + 1, accumulate=True)
    e = rel_l2(whole, host(acc).astype(np.float64))
    say("full bp all views vs sum of one-view calls: rel L2 %.2e" % e)
    assert e <= 1e-6
    x = dev(I.uniform_vector(scan.grid.n_vox, 4061).astype(np.float32).reshape(scan.grid.shape))
    q = host(G.fp(x))
    q1 = np.stack([host(G.fp(x, view_begin=k, view_end=k + 1))[k] for k in range(0, scan.n_views, 17)])
    e = rel_l2(q[::17], q1.astype(np.float64))
    say("full fp all views vs one-view calls: rel L2 %.2e" % e)
    assert e <= 1e-6


def test_posed_large_bp_one_view(torch_cuda):
    """512x1440x256 posed scan, 1024x768 detector: one view FP and BP."""
    cfg = I.config_posed()
    _fp_bp_check(torch_cuda, cfg["scan"], 11, 12, 4031, "posed large view 11")


def _full_size_sart_update(torch, scan, seed, k, lam, label):
    """One weighted SART sub-iteration (Eq. 7) of view k from the prior,
    through the residual and update launches the iteration loop uses, against
    the oracle's sub-iteration on that view.  The update mu1 - mu0 is compared
    with the oracle's rounded to FP32 storage; cells of zero voxel weight stay
    bitwise unchanged.

    Bar: 2e-5 for the column sums (the back-projection's 1e-5 in c and in n,
    plus one-ulp flips of the stored value) plus 1e-7 kappa for the residual.
    From the prior, p - q is a small difference: kappa = |p| / |p - q| (from
    the oracle's own residual norm) multiplies the FP32 rounding of q, and the
    update inherits it."""
    ph = I.industrial_phantom(scan.grid, seed)
    w = ph.weights.astype(np.float32).copy()
    w[:, ::7, :] = 0.0
    prior = ph.prior.astype(np.float32)
    say("%s view %d: oracle" % (label, k))
    pk = ref.Oracle(scan).fp(ph.truth, k, k + 1).astype(np.float32)
    one = I.Scan(scan.grid, scan.views[k:k + 1], scan.det_rows, scan.det_cols, scan.R, scan.T)
    mu_ref, r2 = ref.Oracle(one).sart(pk.astype(np.float64), prior.astype(np.float64), 1, lam,
                                      vox_weights=w.astype(np.float64))
    kappa = float(np.linalg.norm(pk.astype(np.float64)) / math.sqrt(r2[0]))
    tol = 2e-5 + 1e-7 * kappa
    say("%s view %d: gpu" % (label, k))
    G = _geom(scan)
    proj = np.zeros(scan.proj_shape, np.float32)
    proj[k] = pk[0]
    vol = dev(prior)
    ws = torch.empty(G.workspace_bytes(), dtype=torch.uint8, device="cuda")
    G.sart_residual(k, dev(proj), vol, ws)
    G.sart_update(k, vol, ws, lam, vox_weights=dev(w))
    got = host(vol)
    d_got = got.astype(np.float64) - prior
    d_ref = mu_ref.astype(np.float32).astype(np.float64) - prior
    e = rel_l2(d_got, d_ref)
    frozen = w == 0.0
    say("%s: rel L2 of the update %.2e, bar %.2e (kappa %.0f; max %.2e of max |d| %.2e)" %
        (label, e, tol, kappa, np.abs(d_got - d_ref).max(), np.abs(d_ref).max()))
    assert np.count_nonzero(d_ref) > 100000  # the stored update is not trivial
    assert e <= tol
    assert np.array_equal(got[frozen], prior[frozen])


@pytest.mark.parametrize("posed", [False, True])
def test_single_scan_full_size_sart_update(torch_cuda, posed):
    """256x720x128, 512x512 detector, unposed view 37 and posed view 81."""
    cfg = I.config_single()
    scan = cfg["scan"]
    if posed:
        R, T, _ = I.random_pose(2002)
        scan = I.Scan(scan.grid, scan.views, scan.det_rows, scan.det_cols, R, T)
    _full_size_sart_update(torch_cuda, scan, cfg["seed"], 81 if posed else 37, cfg["lam"],
                           "full sart update posed=%s" % posed)


def test_posed_large_sart_update(torch_cuda):
    """512x1440x256 posed scan, 1024x768 detector, view 23."""
    cfg = I.config_posed()
    _full_size_sart_update(torch_cuda, cfg["scan"], cfg["seed"], 23, cfg["lam"], "posed large sart update")


# ------------------------------------------------------------------ SART

def _sart_pair(torch, scan, ph, n_iter, weighted, from_prior, lam=0.5, label=""):
    o = ref.Oracle(scan)
    G = _geom(scan)
    p = o.fp(ph.truth)
    mu0 = ph.prior if from_prior else np.zeros(scan.grid.shape)
    vw = ph.weights if weighted else None
    errs = []
    vol = dev(mu0.astype(np.float32))
    pg = dev(p.astype(np.float32))
    vwg = dev(vw.astype(np.float32)) if vw is not None else None
    mu_ref = mu0.copy()
    for it in range(n_iter):
        say(label, "sart iteration", it)
        G.sart(pg, vol, it + 1, lam, vox_weights=vwg, start_iter=it)
        mu_ref, _ = o.sart(p.astype(np.float32).astype(np.float64), mu_ref, it + 1, lam,
                           vox_weights=vw, start_iter=it)
        errs.append(rel_l2(host(vol), mu_ref))
    say(label, "per-iteration rel L2", " ".join("%.2e" % e for e in errs))
    return errs, host(vol), mu_ref


def test_sart_tiny_ten_iterations(torch_cuda):
    cfg = I.config_tiny()
    scan = cfg["scan"]
    ph = I.tiny_phantom(scan.grid, cfg["seed"])
    errs, got, want = _sart_pair(torch_cuda, scan, ph, 10, False, False, label="tiny")
    assert max(errs) <= 6e-6  # measured 6.0e-7


def test_sart_weighted_prior_posed_scaled(torch_cuda):
    scan = I.scaled_single(n_h=24, n_theta=72, n_r=16, n_views=16, det=48, posed_seed=2006)
    ph = I.industrial_phantom(scan.grid, 1002, n_annuli=5, n_incl=6)
    errs, got, want = _sart_pair(torch_cuda, scan, ph, 3, True, True, label="scaled weighted")
    assert max(errs) <= 1.5e-6  # measured 1.4e-7


@pytest.mark.parametrize("subset", [1, 2])
def test_sart_ragged_detector(torch_cuda, subset):
    """A posed scan on a 13 x 21 detector (neither side a multiple of the 8x8
    residual tiles whose maxima set the update's fixed-point scales): weighted
    SART (subset 1) and ordered subsets of 2 views against the oracle."""
    grid = I.Grid(8, 36, 8, 0.5, 6.0, -3.0, 3.0, 0.05)
    R, T = I.pose_from(0.4, 0.12, 1.1, [0.3, -0.2, 0.1])
    scan = I.Scan(grid, I.circular_views(6, 40.0, 80.0, 0.7, phi0=0.2), 13, 21, R, T)
    ph = I.industrial_phantom(grid, 4040, n_annuli=3, n_incl=3)
    o = ref.Oracle(scan)
    p = o.fp(ph.truth)
    G = _geom(scan)
    pg, wg = dev(p.astype(np.float32)), dev(ph.weights.astype(np.float32))
    vol = dev(ph.prior.astype(np.float32))
    mu = ph.prior.copy()
    for it in range(2):
        say("ragged detector subset %d iteration %d" % (subset, it))
        if subset == 1:
            G.sart(pg, vol, it + 1, 0.5, vox_weights=wg, start_iter=it)
        else:
            G.os_sart(pg, vol, it + 1, subset, 0.5, vox_weights=wg, start_iter=it)
        mu, _ = o.sart(p.astype(np.float32).astype(np.float64), mu, it + 1, 0.5, vox_weights=ph.weights,
                       start_iter=it, subset=subset)
        e = rel_l2(host(vol), mu)
        say("ragged detector subset %d iteration %d rel L2 %.2e" % (subset, it, e))
        assert e <= 5e-7  # measured at most 5.1e-8
    assert rel_l2(mu, ph.prior) > 1e-3  # the updates are not trivial


def test_fine_sectors_partial_edge_table(torch_cuda):
    """A small grid with 1600 sectors (4 x 1600 x 16): its whole sector-edge
    table would crowd the CU, so the back-projection stages only each
    super-block's edges (on 4-block super-blocks, the only ones that stage a
    part of the table).  FP and
    the plain transpose against the oracle (with the adjoint identity), and
    weighted SART for 2 iterations."""
    grid = I.Grid(4, 1600, 16, 1.0, 6.0, -2.0, 2.0, 0.01)
    R, T = I.pose_from(0.3, 0.08, 0.7, [0.2, -0.1, 0.05])
    scan = I.Scan(grid, I.circular_views(4, 40.0, 80.0, 0.5, phi0=0.13), 10, 30, R, T)
    _fp_bp_check(torch_cuda, scan, 0, 4, 4070, "fine sectors")
    rng = np.random.default_rng(4071)
    truth = rng.uniform(0.0, 1.0, size=grid.shape)
    prior = truth * rng.uniform(0.8, 1.2, size=grid.shape)
    wv = rng.uniform(0.25, 1.0, size=grid.shape)
    o = ref.Oracle(scan)
    p = o.fp(truth)
    G = _geom(scan)
    pg, wg = dev(p.astype(np.float32)), dev(wv.astype(np.float32))
    vol = dev(prior.astype(np.float32))
    mu = prior.astype(np.float32).astype(np.float64)
    for it in range(2):
        say("fine sectors sart iteration", it)
        G.sart(pg, vol, it + 1, 0.5, vox_weights=wg, start_iter=it)
        mu, _ = o.sart(p.astype(np.float32).astype(np.float64), mu, it + 1, 0.5, vox_weights=wv.astype(np.float32),
                       start_iter=it)
        e = rel_l2(host(vol), mu)
        say("fine sectors sart iteration %d rel L2 %.2e" % (it, e))
        assert e <= 1.5e-5  # measured at most 1.4e-6
    assert rel_l2(mu, prior) > 1e-3


def _large_grid_check(torch_cuda, scan, seed, label, min_met):
    """FP, transpose and adjoint of a large grid against the oracle on a small
    detector (the bars of every grid), and one weighted SART sub-iteration on
    the cells the oracle meets."""
    grid = scan.grid
    _fp_bp_check(torch_cuda, scan, 0, 3, seed, label)
    # one SART sub-iteration of view 0.  With a few hundred rays for millions
    # of cells most touched cells meet one ray; a ray within FP32 rounding of a cell's face
    # may give that cell a tiny positive length where FP64 gives none, and
    # Eq. 7 then moves it by the ray's whole residual.  So the update is held
    # to 1e-4 on the cells the oracle's view meets (n_m > 0), and the cells
    # changed beyond those are counted.  Measured 3.8e-6 and 3.2e-6.
    o = ref.Oracle(scan)
    x = I.uniform_vector(grid.n_vox, seed + 1).reshape(grid.shape)
    p = o.fp(x)
    prior = (x * 0.9).astype(np.float32)
    G = _geom(scan)
    vol = dev(prior)
    ws = torch_cuda.empty(G.workspace_bytes(), dtype=torch_cuda.uint8, device="cuda")
    say(label + ": sart sub-iteration")
    G.sart_residual(0, dev(p.astype(np.float32)), vol, ws)
    G.sart_update(0, vol, ws, 0.5)
    one = I.Scan(grid, scan.views[:1], scan.det_rows, scan.det_cols, scan.R, scan.T)
    o1 = ref.Oracle(one)
    mu, _ = o1.sart(p[:1].astype(np.float32).astype(np.float64), prior.astype(np.float64), 1, 0.5)
    _, n = o1.bp(np.ones((1, scan.det_rows, scan.det_cols)), colsum=True)
    met = n.reshape(grid.shape) > 0.0
    d_got = host(vol).astype(np.float64) - prior
    d_ref = mu.astype(np.float32).astype(np.float64) - prior
    e = rel_l2(d_got[met], d_ref[met])
    extra = int(np.count_nonzero(d_got[~met]))
    say(label + ": update rel L2 on the %d met cells %.2e, %d more cells changed" % (met.sum(), e, extra))
    assert met.sum() > min_met and e <= 3e-5
    assert extra <= 1e-3 * met.sum()


def test_grid_above_2_25_cells_whole_edge_table(torch_cuda):
    """A 128 x 720 x 400 grid (36.9 M cells, 4-block super-blocks) whose whole
    sector-edge table fits beside them: FP, transpose and adjoint against the
    oracle on a small detector, and one weighted SART iteration.  Its shells
    are 0.025 mm thin: crossings 2.5e-5 mm apart still land in the right
    cells because the walks measure positions from a point next to each
    super-block (measured 2.6e-6 for the back-projection)."""
    grid = I.Grid(128, 720, 400, 0.0, 10.0, -5.0, 5.0)
    assert grid.n_vox > 1 << 25
    scan = I.Scan(grid, I.circular_views(3, 100.0, 200.0, 1.0, phi0=0.3), 12, 20, np.eye(3), np.zeros(3))
    _large_grid_check(torch_cuda, scan, 4080, "grid above 2^25 cells", 100000)


def test_grid_on_8_block_super_blocks(torch_cuda):
    """A 128 x 1024 x 128 grid (16.8 M cells) that takes 8-block super-blocks
    with none to spare (the whole sector-edge table fits and it gives exactly
    2048 of them): the same checks against the oracle as for the 2^25-cell grid,
    on a 16 x 24 detector.  Its 1024 sectors make the arc the thinnest cell
    dimension (0.031 mm at the middle radius, against 0.078 mm rings and
    slabs)."""
    grid = I.Grid(128, 1024, 128, 0.0, 10.0, -5.0, 5.0)
    scan = I.Scan(grid, I.circular_views(3, 100.0, 200.0, 1.0, phi0=0.17), 16, 24, np.eye(3), np.zeros(3))
    _large_grid_check(torch_cuda, scan, 4090, "8-block grid", 50000)


def test_sart_invariants_bitwise(torch_cuda):
    torch = torch_cuda
    scan = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=8, det=40, posed_seed=2007)
    ph = I.industrial_phantom(scan.grid, 55, n_annuli=4, n_incl=3)
    G = _geom(scan)
    truth = dev(ph.truth.astype(np.float32))
    say("invariants: fixed point")
    p = G.fp(truth)
    vol = truth.clone()
    G.sart(p, vol, 2, 0.5, vox_weights=dev(ph.weights.astype(np.float32)))
    assert torch.equal(vol, truth)
    say("invariants: zero weights")
    w = ph.weights.astype(np.float32).copy()
    w[:, :, :3] = 0.0
    prior = dev(ph.prior.astype(np.float32) * 0.5)
    vol = prior.clone()
    G.sart(p, vol, 1, 0.5, vox_weights=dev(w))
    assert torch.equal(vol[:, :, :3], prior[:, :, :3])
    assert not torch.equal(vol[:, :, 3:], prior[:, :, 3:])
    say("invariants: resume and determinism")
    a = prior.clone()
    G.sart(p, a, 4, 0.5)
    b = prior.clone()
    G.sart(p, b, 2, 0.5)
    G.sart(p, b, 4, 0.5, start_iter=2)
    assert torch.equal(a, b)
    e1 = prior.clone()
    G.sart(p, e1, 1, 0.5)
    e2 = prior.clone()
    G.sart(p, e2, 1, 0.5, view_order=np.arange(scan.n_views))
    assert torch.equal(e1, e2)
    e3 = prior.clone()
    G.sart(p, e3, 1, 0.5, view_order=np.arange(scan.n_views)[::-1].copy())
    assert not torch.equal(e1, e3)
    say("invariants: linear in lambda (first view)")
    one = I.Scan(scan.grid, scan.views[:1], scan.det_rows, scan.det_cols, scan.R, scan.T)
    G1 = _geom(one)
    m1 = prior.clone()
    G1.sart(p[:1].contiguous(), m1, 1, 0.25)
    m2 = prior.clone()
    G1.sart(p[:1].contiguous(), m2, 1, 0.5)
    d1 = host(m1) - host(prior)
    d2 = host(m2) - host(prior)
    assert rel_l2(d2, 2 * d1) <= 1e-5


def test_sart_mid_sweep_resume_bitwise(torch_cuda):
    torch = torch_cuda
    scan = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=8, det=40)
    ph = I.industrial_phantom(scan.grid, 56, n_annuli=4, n_incl=3)
    G = _geom(scan)
    p = G.fp(dev(ph.truth.astype(np.float32)))
    prior = dev(ph.prior.astype(np.float32))
    full = prior.clone()
    G.sart(p, full, 2, 0.5)
    # 1 iteration + 3 views, then resume from (1, 3)
    part = prior.clone()
    G.sart(p, part, 1, 0.5)
    first3 = I.Scan(scan.grid, scan.views[:3], scan.det_rows, scan.det_cols, scan.R, scan.T)
    G3 = _geom(first3)
    G3.sart(p[:3].contiguous(), part, 1, 0.5)
    G.sart(p, part, 2, 0.5, start_iter=1, start_view=3)
    assert torch.equal(full, part)


def test_sart_rejects_bad_arguments(torch_cuda):
    from paper_2005_11976_amd import cyl
    scan = I.scaled_single(n_h=8, n_theta=24, n_r=6, n_views=4, det=20)
    G = _geom(scan)
    vol = dev(np.zeros(scan.grid.shape, np.float32))
    p = dev(np.zeros(scan.proj_shape, np.float32))
    tiny_ws = torch_cuda.empty(16, dtype=torch_cuda.uint8, device="cuda")
    with pytest.raises(cyl.CylError, match="workspace"):
        G.sart(p, vol, 1, 0.5, workspace=tiny_ws)
    with pytest.raises(cyl.CylError, match="view_order"):
        G.sart(p, vol, 1, 0.5, view_order=np.array([0, 1, 2, 9]))
    with pytest.raises(cyl.CylError, match="view range"):
        G.fp(vol, p, view_begin=2, view_end=9)


# ------------------------------------------------- rays parallel to the axis

def _axial_scan(kind):
    """Top-down views: each source sits above the grid at (x_k, y_k) and its
    detector lies below it, perpendicular to the object axis, so the ray to
    the central pixel of the odd 9 x 9 detector has d_xy = 0 exactly (all
    coordinates are binary fractions) and runs parallel to the axis; the other
    rays are steep (xy slope at most 1/120).  The sources sit inside sectors
    and rings, away from every boundary.  kind: "plain" (identity pose),
    "shifted" (a binary-fraction shift keeps the central rays exactly axial)
    or "rotated" (a rotation about the axis, after which rounding may leave
    them nearly axial instead)."""
    g = I.Grid(6, 24, 6, 0.0, 6.0, -3.0, 3.0, 0.05)
    p = 0.25
    views = []
    for x, y in [(1.375, 0.625), (-2.125, 1.875), (0.375, -3.375), (-4.625, -1.125)]:
        views.append([x, y, 60.0, x, y, -60.0, p, 0.0, 0.0, 0.0, p, 0.0])
    views = np.array(views, dtype=np.float64)
    R, T = np.eye(3), np.zeros(3)
    if kind == "shifted":
        T = np.array([0.125, -0.25, 0.375])
    elif kind == "rotated":
        R, T = I.pose_from(0.0, 0.0, 0.3, [0.0, 0.0, 0.25])
    return I.Scan(g, views, 9, 9, R, T)


@pytest.mark.parametrize("kind", ["plain", "shifted", "rotated"])
def test_axial_rays_fp_bp_sart(torch_cuda, kind):
    """Rays exactly parallel to the object axis (Eq. 2 and 6, the case where
    the xy direction vanishes): the whole length of the central ray lies in
    one (ring, sector) column.  FP, BP and adjoint against the oracle, and
    weighted SART for 2 iterations."""
    scan = _axial_scan(kind)
    label = "axial " + kind
    o = ref.Oracle(scan)
    if kind != "rotated":
        for k in range(scan.n_views):
            a, e = o.ray_ends(k, 4, 4)
            assert a[0] == e[0] and a[1] == e[1]  # exactly axial in the object frame
    _fp_bp_check(torch_cuda, scan, 0, scan.n_views, 4080, label)
    rng = np.random.default_rng(4081)
    truth = rng.uniform(0.0, 1.0, size=scan.grid.shape)
    prior = truth * rng.uniform(0.8, 1.2, size=scan.grid.shape)
    wv = rng.uniform(0.25, 1.0, size=scan.grid.shape)
    p = o.fp(truth)
    G = _geom(scan)
    pg, wg = dev(p.astype(np.float32)), dev(wv.astype(np.float32))
    vol = dev(prior.astype(np.float32))
    mu = prior.astype(np.float32).astype(np.float64)
    for it in range(2):
        say(label, "sart iteration", it)
        G.sart(pg, vol, it + 1, 0.5, vox_weights=wg, start_iter=it)
        mu, _ = o.sart(p.astype(np.float32).astype(np.float64), mu, it + 1, 0.5, vox_weights=wv.astype(np.float32),
                       start_iter=it)
        e = rel_l2(host(vol), mu)
        say(label, "sart iteration %d rel L2 %.2e" % (it, e))
        assert e <= 1e-5  # measured at most 1.1e-6
    assert rel_l2(mu, prior) > 1e-3


# ------------------------------------- whole SART iterations on the full grids

def _full_grid_sart(torch, scan, truth, prior, weights, data, n_iter, lam, label, tols):
    """Weighted SART from the prior over every view of `scan`, the launches
    the bench times (cyl_sart_run), against the oracle's iterates after each
    iteration."""
    G = _geom(scan)
    pg = dev(data.astype(np.float32))
    wg = dev(weights.astype(np.float32))
    vol = dev(prior.astype(np.float32))
    mu = prior.astype(np.float32).astype(np.float64)
    errs = []
    for it in range(n_iter):
        say(label, "gpu iteration", it)
        G.sart(pg, vol, it + 1, lam, vox_weights=wg, start_iter=it)
        # the oracle's sweep, one view at a time (a sub-iteration of Eq. 7
        # depends only on the volume the previous one left)
        for k in range(scan.n_views):
            say(label, "oracle iteration %d view %d" % (it, k))
            one = I.Scan(scan.grid, scan.views[k:k + 1], scan.det_rows, scan.det_cols, scan.R, scan.T)
            mu, _ = ref.Oracle(one).sart(data[k:k + 1].astype(np.float32).astype(np.float64), mu, 1, lam,
                                         vox_weights=weights.astype(np.float32))
        got = host(vol)
        errs.append(rel_l2(got, mu))
        say(label, "iteration %d: rel L2 vs oracle %.3e, max abs %.3e of max, update size %.3e" %
            (it, errs[-1], abs_rel(got, mu), rel_l2(mu, prior)))
    for e, t in zip(errs, tols):
        assert e <= t
    assert rel_l2(mu, prior) > 1e-4  # the iterations move the volume
    return errs


@pytest.mark.timeout(900)
def test_single_scan_full_grid_sart_two_iterations(torch_cuda):
    """256x720x128 grid, full 512 x 512 detector, 12 evenly spaced of the 120
    views (every 10th), weighted SART from the prior for 2 whole iterations,
    compared with the oracle after each (Eq. 7)."""
    cfg = I.config_single()
    s0 = cfg["scan"]
    scan = I.Scan(s0.grid, s0.views[::10], s0.det_rows, s0.det_cols, s0.R, s0.T)
    ph = I.industrial_phantom(scan.grid, cfg["seed"])
    say("full grid sart 256x720x128: oracle data")
    data = ref.Oracle(scan).fp(ph.truth)
    _full_grid_sart(torch_cuda, scan, ph.truth, ph.prior, ph.weights, data, 2, cfg["lam"],
                    "full grid sart 256x720x128", (1e-6, 1e-6))  # measured 6.4e-8, 1.1e-7


@pytest.mark.timeout(900)
def test_posed_large_full_grid_sart_three_views(torch_cuda):
    """512x1440x256 posed grid, full 1024 x 768 detector, 3 views (0, 20, 40)
    with Poisson data at 1e4 photons, one weighted SART iteration from the
    prior against the oracle's."""
    cfg = I.config_posed()
    s0 = cfg["scan"]
    scan = I.Scan(s0.grid, s0.views[[0, 20, 40]], s0.det_rows, s0.det_cols, s0.R, s0.T)
    ph = I.industrial_phantom(scan.grid, cfg["seed"])
    say("full grid sart 512x1440x256 posed: oracle data")
    clean = ref.Oracle(scan).fp(ph.truth)
    data = I.poisson_line_integrals(clean, cfg["photons"], cfg["noise_seed"])
    _full_grid_sart(torch_cuda, scan, ph.truth, ph.prior, ph.weights, data, 1, cfg["lam"],
                    "full grid sart 512x1440x256 posed", (1.5e-5,))  # measured 1.5e-6
