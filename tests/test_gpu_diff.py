"""cyl_fp_diff and cyl_add, and the difference form of SART from a prior.

SART (Eq. 7) is affine in the volume and the data: started from mu0 on data p
it equals mu0 + (SART started from 0 on d = p - A mu0).  The serving path uses
that form so FP16 storage holds small differences; here it is checked in FP32
against the plain form, and the two new entry points against the oracle and
host arithmetic.
"""
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


def test_fp_diff_against_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    scan = I.scaled_single(n_h=16, n_theta=48, n_r=12, n_views=5, det=40, posed_seed=2008)
    G = cyl.Geometry(scan, 0)
    o = ref.Oracle(scan)
    x = (0.02 * I.uniform_vector(scan.grid.n_vox, 4201)).astype(np.float32).reshape(scan.grid.shape)
    base = I.uniform_vector(scan.n_views * scan.det_rows * scan.det_cols, 4202).astype(np.float32)
    base = base.reshape(scan.proj_shape)
    ax = o.fp(x.astype(np.float64))
    want = base.astype(np.float64) - ax
    say("fp_diff f32")
    got = host(G.fp_diff(dev(x), dev(base)))
    e = float(np.linalg.norm(got - want) / np.linalg.norm(ax))
    say("fp_diff error relative to |A x|: %.2e" % e)
    assert e <= 1e-5
    # views subrange, in place on the base buffer, FP16 output of an FP32 difference
    b = dev(base)
    G.fp_diff(dev(x), b, out=b, view_begin=1, view_end=3)
    hb = host(b)
    assert np.array_equal(hb[0], base[0].astype(np.float64)) and np.array_equal(hb[3:], base[3:].astype(np.float64))
    assert float(np.linalg.norm(hb[1:3] - want[1:3]) / np.linalg.norm(ax[1:3])) <= 1e-5
    say("fp_diff -> f16")
    g16 = host(G.fp_diff(dev(x), dev(base), out_dtype=torch.float16))
    assert np.all(np.abs(g16 - want) <= 2.0 ** -11 * np.abs(want) * 1.001 + 1e-5 * np.abs(ax).max())


def test_add_storage_types(torch_cuda):
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    rng = np.random.default_rng(4203)
    a = rng.standard_normal(100003).astype(np.float32)
    b = rng.standard_normal(100003).astype(np.float32)
    got = host(cyl.add(dev(a), dev(b)))
    assert np.array_equal(got, (a + b).astype(np.float64))
    a16 = dev(a, torch.float16)
    got16 = cyl.add(a16, dev(b), out=torch.empty_like(a16))
    want16 = (host(a16).astype(np.float32) + b).astype(np.float16).astype(np.float64)
    assert np.array_equal(host(got16), want16)
    cyl.add(dev(a[:0]), dev(b[:0]))


def test_difference_form_of_sart(torch_cuda):
    """SART from the prior on p == prior + SART from 0 on p - A prior (FP32,
    up to rounding), and both against the oracle."""
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    scan = I.scaled_single(n_h=24, n_theta=72, n_r=16, n_views=16, det=48, posed_seed=2006)
    ph = I.industrial_phantom(scan.grid, 1006, n_annuli=5, n_incl=6)
    G = cyl.Geometry(scan, 0)
    o = ref.Oracle(scan)
    p = o.fp(ph.truth).astype(np.float32)
    prior = ph.prior.astype(np.float32)
    w = dev(ph.weights.astype(np.float32))
    say("plain form")
    vol = dev(prior)
    G.sart(dev(p), vol, 2, 0.5, vox_weights=w)
    say("difference form")
    d = G.fp_diff(dev(prior), dev(p))
    delta = torch.zeros_like(vol)
    G.sart(d, delta, 2, 0.5, vox_weights=w)
    mu = cyl.add(dev(prior), delta)
    e = rel_l2(host(mu), host(vol))
    want, _ = o.sart(p.astype(np.float64), prior.astype(np.float64), 2, 0.5,
                     vox_weights=ph.weights.astype(np.float32).astype(np.float64))
    say("difference vs plain form %.2e; vs oracle %.2e / %.2e" % (e, rel_l2(host(mu), want),
                                                                   rel_l2(host(vol), want)))
    assert e <= 1e-5
    assert rel_l2(host(mu), want) <= 1e-4
