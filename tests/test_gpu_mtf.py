"""MTF on the GPU (Sec. 2.3, Eq. 8): cyl_mtf against the reference
measurement bit for bit (FP32/FP16/BF16 volumes, odd and even slice counts,
per ring and per window), and a small version of the whole experiment (line
phantom on a fine grid -> cyl_fp -> SART on a coarser grid -> cyl_mtf)
against the same chain run by the FP64 oracle."""
import numpy as np
import pytest

from oracle import mtf as M
from oracle import ref
from paper_2005_11976_amd import inputs as I
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_11976_amd import cyl
    cyl.lib()
    return torch


@pytest.mark.parametrize("dtype_name", ["float32", "float16", "bfloat16"])
@pytest.mark.parametrize("n_h", [4, 5])
def test_mtf_kernel_matches_reference(torch_cuda, dtype_name, n_h):
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    rng = np.random.default_rng(4600 + n_h)
    vol = rng.uniform(0.0, 0.05, size=(n_h, 37, 23)).astype(np.float32)
    vol[:, :, 7] = 0.0  # a ring of zeros: modulation 0 by definition
    v = dev(vol, getattr(torch, dtype_name))
    hv = host(v).reshape(vol.shape)  # the values the kernel sees, in FP64
    say("mtf kernel", dtype_name, n_h)
    got = host(cyl.mtf(v, 0))
    assert np.array_equal(got, M.mtf_azimuthal(hv))
    assert got[7] == 0.0
    for w in (1, 5, 23):
        assert np.array_equal(host(cyl.mtf(v, w)), M.mtf_radial(hv, w)), w
    with pytest.raises(cyl.CylError, match="window"):
        cyl.mtf(v, 24)


def _small_mtf_scans(n_views=24):
    fine = I.Grid(8, 96, 32, 0.0, 10.0, -0.8, 0.8)
    coarse = I.Grid(8, 48, 32, 0.0, 10.0, -0.8, 0.8)
    views = I.circular_views(n_views, 80.0, 160.0, 0.2)  # the sample fits the 256 x 24 detector
    return (I.Scan(fine, views, 24, 256, *I.identity_pose()),
            I.Scan(coarse, views, 24, 256, *I.identity_pose()))


@pytest.mark.parametrize("kind", ["azimuthal", "radial"])
def test_small_mtf_chain_matches_oracle_chain(torch_cuda, kind):
    from paper_2005_11976_amd import cyl
    fine, coarse = _small_mtf_scans()
    n_l = 4
    ph = I.line_phantom(fine.grid, kind, n_l)
    say("mtf chain", kind)
    p = cyl.Geometry(fine, 0).fp(dev(ph.astype(np.float32)))
    vol = dev(np.zeros(coarse.grid.shape, np.float32))
    cyl.Geometry(coarse, 0).sart(p, vol, 3, 0.5, nonneg=True)
    ring = host(cyl.mtf(vol, 0))
    win = host(cyl.mtf(vol, 32 // n_l))
    o_p = ref.Oracle(fine).fp(ph)
    o_vol, _ = ref.Oracle(coarse).sart(o_p, np.zeros(coarse.grid.shape), 3, 0.5, nonneg=True)
    o_ring = M.mtf_azimuthal(o_vol)
    o_win = M.mtf_radial(o_vol, 32 // n_l)
    say("mtf chain %s: ring max diff %.2e, window max diff %.2e, slice m %.4f"
        % (kind, np.abs(ring - o_ring).max(), np.abs(win - o_win).max(), M.mtf_slice(o_vol)))
    assert np.abs(ring - o_ring).max() <= 1e-4
    assert np.abs(win - o_win).max() <= 1e-4
    assert M.mtf_slice(o_vol) > 0.2  # the lines are resolved at this frequency
