"""The paper's own projector pair on the GPU (cyl_fp_sampled, cyl_bp_voxel,
cyl_sart_run_sampled; Sec. 2.2) against its FP64 reference
(oracle/sampled.py).  Bars: trilinear sampling and the voxel-driven
back-projection within 2e-5 relative L2 (FP32 sample positions and an FP32
projection of the cell centres); nearest sampling within 1e-4 (a sample
within rounding of a cell face may land in either cell); SART with the pair
within 1e-4 per iteration."""
import numpy as np
import pytest

from oracle import sampled as S
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


def _scan(posed):
    grid = I.Grid(6, 24, 8, 0.5, 6.0, -2.0, 2.0, 0.2)
    views = I.circular_views(5, 40.0, 80.0, 0.6, phi0=0.3)
    R, T = I.pose_from(0.4, 0.15, 1.1, [0.3, -0.2, 0.1]) if posed else I.identity_pose()
    return I.Scan(grid, np.asarray(views, dtype=np.float64), 14, 26, R, T)


@pytest.mark.parametrize("posed", [False, True])
@pytest.mark.parametrize("interp", [0, 1])
def test_fp_sampled_matches_reference(torch_cuda, posed, interp):
    from paper_2005_11976_amd import cyl
    scan = _scan(posed)
    vol = np.random.default_rng(4800).uniform(0.0, 1.0, size=scan.grid.shape)
    step = 0.07
    say("fp sampled", posed, interp)
    got = host(cyl.Geometry(scan, 0).fp_sampled(dev(vol.astype(np.float32)), step, interp))
    want, _ = S.sampled_fp(scan, vol, step, "linear" if interp else "nearest")
    e = rel_l2(got, want)
    say("fp sampled posed=%s interp=%d rel L2 %.2e" % (posed, interp, e))
    assert e <= (2e-5 if interp else 1e-4)


@pytest.mark.parametrize("posed", [False, True])
def test_bp_voxel_matches_reference(torch_cuda, posed):
    from paper_2005_11976_amd import cyl
    scan = _scan(posed)
    y = np.random.default_rng(4801).uniform(-1.0, 1.0, size=scan.proj_shape)
    G = cyl.Geometry(scan, 0)
    say("bp voxel", posed)
    got = host(G.bp_voxel(dev(y.astype(np.float32)), view_begin=1, view_end=4))
    want, _ = S.voxel_bp(scan, y[1:4], 1, 4)
    e = rel_l2(got, want)
    say("bp voxel posed=%s rel L2 %.2e" % (posed, e))
    assert e <= 2e-5
    # accumulate adds onto what is there
    base = dev(np.full(scan.grid.shape, 0.5, np.float32))
    G.bp_voxel(dev(y.astype(np.float32)), base, view_begin=1, view_end=4, accumulate=True)
    assert rel_l2(host(base), want + 0.5) <= 2e-5


def test_sampled_sart_matches_reference(torch_cuda):
    from paper_2005_11976_amd import cyl
    scan = _scan(True)
    ph = I.industrial_phantom(scan.grid, 4802, n_annuli=3, n_incl=2)
    step = 0.07
    p, _ = S.sampled_fp(scan, ph.truth, step, "linear")
    G = cyl.Geometry(scan, 0)
    vol = dev(ph.prior.astype(np.float32))
    pg = dev(p.astype(np.float32))
    wg = dev(ph.weights.astype(np.float32))
    mu = ph.prior.copy()
    for it in range(2):
        say("sampled sart iteration", it)
        G.sart_sampled(pg, vol, it + 1, step, 1, 0.5, vox_weights=wg, start_iter=it)
        mu = S.sampled_sart(scan, p.astype(np.float32).astype(np.float64), mu, 1, step, "linear", 0.5,
                            vox_weights=ph.weights)
        e = rel_l2(host(vol), mu)
        say("sampled sart iteration %d rel L2 %.2e" % (it, e))
        assert e <= 1e-4
    assert rel_l2(mu, ph.prior) > 1e-3  # the updates are not trivial


def test_sampled_rejects_bad_arguments(torch_cuda):
    from paper_2005_11976_amd import cyl
    scan = _scan(False)
    G = cyl.Geometry(scan, 0)
    vol = dev(np.zeros(scan.grid.shape, np.float32))
    with pytest.raises(cyl.CylError, match="step"):
        G.fp_sampled(vol, 0.0)
    with pytest.raises(cyl.CylError, match="step"):
        G.fp_sampled(vol, 1e-12)
    with pytest.raises(cyl.CylError, match="interp"):
        G.fp_sampled(vol, 0.1, 2)
    with pytest.raises(cyl.CylError, match="view range"):
        G.bp_voxel(dev(np.zeros(scan.proj_shape, np.float32)), view_begin=3, view_end=9)
