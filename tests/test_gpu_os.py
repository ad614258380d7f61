"""Ordered-subset SART on the GPU (cyl_os_sart_run; Eq. 7 with an ordered
subset of several projections, up to SIRT) against the FP64 oracle's
ordered-subset SART: relative L2 of every iterate <= 1e-4, as for the
one-projection sweep.  Subset 1 equals cyl_sart_run bit for bit; resume at a
group boundary is bitwise; bad subsets and resume points are rejected."""
import numpy as np
import pytest

from oracle import ref
from paper_2005_11976_amd import inputs as I
from tests.gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu


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


def _os_pair(scan, ph, n_iter, subset, weighted, from_prior, order=None, lam=0.5, label=""):
    o = ref.Oracle(scan)
    G = _geom(scan)
    p = o.fp(ph.truth)
    mu0 = ph.prior if from_prior else np.zeros(scan.grid.shape)
    vw = ph.weights if weighted else None
    vol = dev(mu0.astype(np.float32))
    pg = dev(p.astype(np.float32))
    vwg = dev(vw.astype(np.float32)) if vw is not None else None
    mu_ref = mu0.copy()
    errs = []
    for it in range(n_iter):
        say(label, "os-sart iteration", it, "subset", subset)
        G.os_sart(pg, vol, it + 1, subset, lam, vox_weights=vwg, view_order=order, start_iter=it)
        mu_ref, _ = o.sart(p.astype(np.float32).astype(np.float64), mu_ref, it + 1, lam, vox_weights=vw,
                           view_order=order, start_iter=it, subset=subset)
        errs.append(rel_l2(host(vol), mu_ref))
    say(label, "per-iteration rel L2", " ".join("%.2e" % e for e in errs))
    return errs


@pytest.mark.parametrize("subset", [3, 32])
def test_os_tiny_matches_oracle(torch_cuda, subset):
    cfg = I.config_tiny()
    scan = cfg["scan"]
    ph = I.tiny_phantom(scan.grid, cfg["seed"])
    errs = _os_pair(scan, ph, 6, subset, False, False, label="tiny")
    assert max(errs) <= 1.5e-5  # measured at most 1.5e-6


def test_os_weighted_posed_ragged_groups_matches_oracle(torch_cuda):
    """16 views in groups of 5 (5, 5, 5, 1) in a permuted order, voxel weights,
    from the prior, posed object."""
    scan = I.scaled_single(n_h=24, n_theta=72, n_r=16, n_views=16, det=48, posed_seed=2006)
    ph = I.industrial_phantom(scan.grid, 1002, n_annuli=5, n_incl=6)
    order = np.random.default_rng(4410).permutation(scan.n_views).astype(np.int32)
    errs = _os_pair(scan, ph, 3, 5, True, True, order=order, label="scaled weighted os5")
    assert max(errs) <= 7e-7  # measured 6.7e-8


def test_sirt_scaled_matches_oracle(torch_cuda):
    scan = I.scaled_single(n_h=32, n_theta=96, n_r=24, n_views=24, det=64)
    ph = I.industrial_phantom(scan.grid, 1003, n_annuli=5, n_incl=6)
    errs = _os_pair(scan, ph, 3, scan.n_views, True, True, label="scaled sirt")
    assert max(errs) <= 3e-7  # measured 2.9e-8


def test_os_subset_one_is_sart_and_resume_bitwise(torch_cuda):
    torch = torch_cuda
    scan = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=8, det=40, posed_seed=2007)
    ph = I.industrial_phantom(scan.grid, 57, n_annuli=4, n_incl=3)
    G = _geom(scan)
    p = G.fp(dev(ph.truth.astype(np.float32)))
    prior = dev(ph.prior.astype(np.float32))
    w = dev(ph.weights.astype(np.float32))
    say("os: subset 1 against the one-projection sweep")
    a = prior.clone()
    G.sart(p, a, 2, 0.5, vox_weights=w)
    b = prior.clone()
    G.os_sart(p, b, 2, 1, 0.5, vox_weights=w)
    assert torch.equal(a, b)
    say("os: resume at a group boundary, determinism")
    full = prior.clone()
    G.os_sart(p, full, 2, 3, 0.5, vox_weights=w)
    again = prior.clone()
    G.os_sart(p, again, 2, 3, 0.5, vox_weights=w)
    assert torch.equal(full, again)
    part = prior.clone()
    G.os_sart(p, part, 1, 3, 0.5, vox_weights=w)
    first = I.Scan(scan.grid, scan.views[:3], scan.det_rows, scan.det_cols, scan.R, scan.T)
    _geom(first).os_sart(p[:3].contiguous(), part, 1, 3, 0.5, vox_weights=w)
    G.os_sart(p, part, 2, 3, 0.5, vox_weights=w, start_iter=1, start_view=3)
    assert torch.equal(full, part)
    say("os: a subset larger than the scan is SIRT")
    s1 = prior.clone()
    G.os_sart(p, s1, 1, scan.n_views, 0.5)
    s2 = prior.clone()
    G.os_sart(p, s2, 1, 1000, 0.5)
    assert torch.equal(s1, s2)
    assert not torch.equal(s1, a)


def test_os_rejects_bad_arguments(torch_cuda):
    from paper_2005_11976_amd import cyl
    scan = I.scaled_single(n_h=8, n_theta=24, n_r=6, n_views=6, det=20)
    G = _geom(scan)
    vol = dev(np.zeros(scan.grid.shape, np.float32))
    p = dev(np.zeros(scan.proj_shape, np.float32))
    with pytest.raises(cyl.CylError, match="subset"):
        G.os_sart(p, vol, 1, 0, 0.5)
    with pytest.raises(cyl.CylError, match="boundary"):
        G.os_sart(p, vol, 1, 4, 0.5, start_view=2)
    small = torch_cuda.empty(G.os_workspace_bytes(2) - 1, dtype=torch_cuda.uint8, device="cuda")
    with pytest.raises(cyl.CylError, match="workspace"):
        G.os_sart(p, vol, 1, 4, 0.5, workspace=small)
