"""cyl_sart_run_static (the entry point that allocates nothing) against
cyl_sart_run on the same inputs: the same kernels, so the results must be
bitwise equal.  Two calls in a row, the second on a smaller scan, so the
static scratch is reused with the first call's contents still in it; a third
call on a geometry whose workspace exceeds the scratch is refused."""
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


def _case(scan, seed):
    ph = I.industrial_phantom(scan.grid, seed, n_annuli=3, n_incl=3)
    p = ref.Oracle(scan).fp(ph.truth)
    return ph, p


def _run_both(torch, scan, seed, n_iter, label):
    from paper_2005_11976_amd import cyl
    ph, p = _case(scan, seed)
    G = cyl.Geometry(scan, 0)
    pg = dev(p.astype(np.float32))
    wg = dev(ph.weights.astype(np.float32))
    a = dev(ph.prior.astype(np.float32))
    b = a.clone()
    say(label, "cyl_sart_run", scan.grid.shape, scan.proj_shape)
    G.sart(pg, a, n_iter, 0.5, vox_weights=wg)
    say(label, "cyl_sart_run_static")
    G.sart_static(pg, b, n_iter, 0.5, vox_weights=wg)
    ha, hb = host(a), host(b)
    say(label, "rel L2 static vs workspace %.3e, max abs %.3e" % (rel_l2(hb, ha), float(np.abs(hb - ha).max())))
    assert np.array_equal(ha, hb)
    # and the pair is the oracle's SART (the bar of the single-scan parity tests)
    mu, _ = ref.Oracle(scan).sart(p.astype(np.float32).astype(np.float64), ph.prior.astype(np.float32), n_iter,
                                  0.5, vox_weights=ph.weights.astype(np.float32))
    e = rel_l2(hb, mu)
    say(label, "static vs oracle rel L2 %.3e" % e)
    assert e <= 1e-4
    return G


def test_static_scratch_matches_workspace_twice(torch_cuda):
    big = I.scaled_single(n_h=24, n_theta=72, n_r=16, n_views=12, det=96, posed_seed=2006)
    small = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=8, det=40)
    _run_both(torch_cuda, big, 1101, 2, "static-big")
    _run_both(torch_cuda, small, 1102, 2, "static-small")


def test_static_scratch_rejects_oversized_detector(torch_cuda):
    from paper_2005_11976_amd import cyl
    g = I.Grid(4, 16, 4, 0.0, 5.0, -5.0, 5.0)
    scan = I.Scan(g, I.circular_views(2, 50.0, 100.0, 0.01), 1024, 1032, np.eye(3), np.zeros(3))
    G = cyl.Geometry(scan, 0)
    assert G.workspace_bytes() > cyl.SART_STATIC_SCRATCH_BYTES
    p = torch_cuda.zeros(scan.proj_shape, dtype=torch_cuda.float32, device="cuda")
    vol = torch_cuda.zeros(g.shape, dtype=torch_cuda.float32, device="cuda")
    with pytest.raises(cyl.CylError, match="static"):
        G.sart_static(p, vol, 1)
