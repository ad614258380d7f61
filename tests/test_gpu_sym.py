"""Precomputed system matrix for unposed scans (cyl_sym_*): view 0's exact
rows reused for every view through a theta shift.  Checks: projections
against the FP64 oracle (<= 1e-5) and against cyl_fp (<= 1e-6, the same
lengths summed in another order); SART iterates against the oracle's
(<= 1e-4) and against cyl_sart_run (<= 1e-5); bitwise determinism; refusal
of posed scans and of view steps that are not whole sectors; one full view of
the 256x720x128 scan against cyl_fp."""
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


def _scan(n_views=24, posed_seed=None, phi0=0.0):
    s = I.scaled_single(n_h=16, n_theta=96, n_r=16, n_views=n_views, det=56, posed_seed=posed_seed)
    if phi0:
        views = I.circular_views(n_views, 200.0, 400.0, 0.2 * 512 / 56, phi0=phi0)
        s = I.Scan(s.grid, views, s.det_rows, s.det_cols, s.R, s.T)
    return s


@pytest.mark.parametrize("phi0", [0.0, 0.37])
def test_sym_fp_matches_oracle_and_cyl_fp(torch_cuda, phi0):
    from paper_2005_11976_amd import cyl
    scan = _scan(phi0=phi0)
    G = cyl.Geometry(scan, 0)
    say("sym fp", phi0)
    S = cyl.SymMatrix(G)
    assert S.nnz > 0
    x = I.uniform_vector(scan.grid.n_vox, 4900).reshape(scan.grid.shape)
    xg = dev(x.astype(np.float32))
    got = host(S.fp(xg))
    want = ref.Oracle(scan).fp(x.astype(np.float32).astype(np.float64))
    e_o, e_g = rel_l2(got, want), rel_l2(got, host(G.fp(xg)))
    say("sym fp phi0=%.2f: vs oracle %.2e, vs cyl_fp %.2e, nnz %d" % (phi0, e_o, e_g, S.nnz))
    assert e_o <= 1e-5 and e_g <= 1e-6


def test_sym_sart_matches_oracle_and_is_deterministic(torch_cuda):
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    scan = _scan()
    ph = I.industrial_phantom(scan.grid, 4901, n_annuli=4, n_incl=4)
    o = ref.Oracle(scan)
    p = o.fp(ph.truth)
    G = cyl.Geometry(scan, 0)
    S = cyl.SymMatrix(G)
    pg, wg = dev(p.astype(np.float32)), dev(ph.weights.astype(np.float32))
    vol = dev(ph.prior.astype(np.float32))
    mu = ph.prior.copy()
    for it in range(2):
        say("sym sart iteration", it)
        S.sart(pg, vol, it + 1, 0.5, vox_weights=wg, start_iter=it)
        mu, _ = o.sart(p.astype(np.float32).astype(np.float64), mu, it + 1, 0.5, vox_weights=ph.weights,
                       start_iter=it)
        e = rel_l2(host(vol), mu)
        say("sym sart iteration %d vs oracle %.2e" % (it, e))
        assert e <= 1e-4
    gen = dev(ph.prior.astype(np.float32))
    G.sart(pg, gen, 2, 0.5, vox_weights=wg)
    assert rel_l2(host(vol), host(gen)) <= 1e-5
    again = dev(ph.prior.astype(np.float32))
    S.sart(pg, again, 2, 0.5, vox_weights=wg)
    assert torch.equal(again, vol)


def test_sym_refuses_posed_and_off_sector_views(torch_cuda):
    from paper_2005_11976_amd import cyl
    for scan in (_scan(posed_seed=2008), _scan(n_views=7)):
        G = cyl.Geometry(scan, 0)
        with pytest.raises(cyl.CylError, match="rotated"):
            cyl.SymMatrix(G)


def test_sym_full_view_of_the_single_scan(torch_cuda):
    from paper_2005_11976_amd import cyl
    cfg = I.config_single()
    scan = cfg["scan"]
    ph = I.industrial_phantom(scan.grid, cfg["seed"])
    G = cyl.Geometry(scan, 0)
    say("sym full-size build")
    S = cyl.SymMatrix(G)
    t = dev(ph.truth.astype(np.float32))
    got = host(S.fp(t, view_begin=37, view_end=38))[37]
    want = host(G.fp(t, view_begin=37, view_end=38))[37]
    e = rel_l2(got, want)
    say("sym full view 37: vs cyl_fp %.2e, nnz %d" % (e, S.nnz))
    assert e <= 1e-6
