"""Batched SART sub-iterations (cyl_sart_batch_step) against the same scans run
alone.

A batch runs the kernels of the single-scan path with several scans per launch;
each scan's piece split, tile order and block order depend on its own geometry
only, so a scan's result must be bitwise the same alone and in any mix.  The
single-scan path itself is checked against the FP64 oracle elsewhere; here one
mixed run is also compared with the oracle directly.
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


def _scans():
    R, T = I.pose_from(0.4, 0.3, 1.1, [0.7, -0.4, 0.5])
    return [
        ("tiny", I.config_tiny()["scan"]),
        ("scaled_posed", I.scaled_single(n_h=24, n_theta=72, n_r=16, n_views=12, det=48, posed_seed=2006)),
        ("hollow_posed", I.Scan(I.Grid(4, 8, 4, 1.5, 6.0, -2.0, 4.0, 0.3),
                                I.circular_views(5, 40.0, 80.0, 1.1, 0.9, phi0=0.17), 8, 6, R, T)),
        ("ragged", I.Scan(I.Grid(7, 37, 19, 0.0, 6.0, -3.0, 3.0),
                          I.circular_views(7, 40.0, 80.0, 1.1, 0.9, phi0=0.3), 13, 21, np.eye(3), np.zeros(3))),
    ]


class _Job:
    def __init__(self, torch, name, scan, seed, tdt, n_iter):
        from paper_2005_11976_amd import cyl
        self.name, self.scan, self.n_iter = name, scan, n_iter
        self.G = cyl.Geometry(scan, 0)
        ph = I.industrial_phantom(scan.grid, seed, n_annuli=3, n_incl=3) if scan.grid.n_theta >= 16 \
            else None
        if ph is None:
            truth = 0.02 * I.uniform_vector(scan.grid.n_vox, seed).reshape(scan.grid.shape)
            prior = truth * 0.9
            w = np.ones(scan.grid.shape)
        else:
            truth, prior, w = ph.truth, ph.prior, ph.weights
        o = ref.Oracle(scan)
        self.p_host = o.fp(truth)
        self.prior_host, self.w_host = prior, w
        self.p = dev(self.p_host.astype(np.float32), tdt)
        self.w = dev(w.astype(np.float32), tdt)
        self.vol = dev(prior.astype(np.float32), tdt)
        self.ws = torch.empty(self.G.workspace_bytes(), dtype=torch.uint8, device="cuda")
        self.cursor = 0

    @property
    def done(self):
        return self.cursor >= self.n_iter * self.scan.n_views

    def entry(self):
        from paper_2005_11976_amd import cyl
        return cyl.BatchEntry(self.G, self.cursor % self.scan.n_views, self.p, self.vol, self.ws,
                              vox_weights=self.w, lam=0.5)


def _alone(torch, job):
    vol = job.vol.clone()
    job.G.sart(job.p, vol, job.n_iter, 0.5, vox_weights=job.w, workspace=job.ws)
    return vol


def _batched(jobs, order_seed):
    """Continuous batching: every step takes each unfinished job's next view;
    jobs join at staggered steps and leave when done."""
    from paper_2005_11976_amd import cyl
    rng = np.random.default_rng(order_seed)
    join = {id(j): int(rng.integers(0, 5)) for j in jobs}
    step = 0
    while not all(j.done for j in jobs):
        active = [j for j in jobs if not j.done and join[id(j)] <= step]
        rng.shuffle(active)
        if active:
            cyl.sart_batch_step([j.entry() for j in active])
            for j in active:
                j.cursor += 1
        step += 1


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_batch_matches_alone_bitwise(torch_cuda, dtype_name):
    torch = torch_cuda
    tdt = getattr(torch, dtype_name)
    jobs = [_Job(torch, n, s, 1100 + i, tdt, 2) for i, (n, s) in enumerate(_scans())]
    # a second scan on the same geometry with other data
    jobs.append(_Job(torch, "tiny_b", jobs[0].scan, 1199, tdt, 3))
    alone = []
    for j in jobs:
        say("alone", j.name, dtype_name)
        alone.append(host(_alone(torch, j)))
    say("batched", dtype_name)
    _batched(jobs, 7)
    for j, a in zip(jobs, alone):
        got = host(j.vol)
        say("batched vs alone", j.name, "max |diff| %.3g" % float(np.max(np.abs(got - a))))
        assert np.array_equal(got, a), j.name


def test_batch_mixing_super_block_sizes_matches_alone_bitwise(torch_cuda):
    """A grid just above 2^25 cells and two small ones (back-projected on
    4-block super-blocks) batched with a 128 x 1024 x 128 grid (8-block
    super-blocks: the whole sector-edge table fits and it has 2048 of them):
    the step launches each size separately, and every scan's result is
    bitwise its result alone."""
    torch = torch_cuda
    views = I.circular_views(3, 100.0, 200.0, 0.8, phi0=0.21)
    big = I.Scan(I.Grid(64, 1024, 513, 0.0, 10.0, -5.0, 5.0), views, 20, 28, np.eye(3), np.zeros(3))
    assert big.grid.n_vox > 1 << 25
    mid = I.Scan(I.Grid(128, 1024, 128, 0.0, 10.0, -5.0, 5.0), views, 20, 28, np.eye(3), np.zeros(3))
    scans = [("big", big), ("mid", mid), ("scaled_posed", _scans()[1][1]), ("tiny", _scans()[0][1])]
    jobs = [_Job(torch, n, s, 1400 + i, torch.float32, 1) for i, (n, s) in enumerate(scans)]
    alone = []
    for j in jobs:
        say("alone", j.name)
        alone.append(host(_alone(torch, j)))
    say("batched, mixed super-block sizes")
    _batched(jobs, 13)
    for j, a in zip(jobs, alone):
        got = host(j.vol)
        say("mixed batch vs alone", j.name, "max |diff| %.3g" % float(np.max(np.abs(got - a))))
        assert np.array_equal(got, a), j.name
        assert not np.array_equal(got, j.prior_host.astype(np.float32)), j.name  # updated


def test_batch_of_more_than_16_and_oracle(torch_cuda):
    """18 tiny scans in one step call (two launches of 16 and 2), one step per
    view for one iteration; every result against the FP64 oracle's SART."""
    torch = torch_cuda
    base = I.config_tiny()["scan"]
    jobs = [_Job(torch, "tiny%d" % i, base, 1300 + i, torch.float32, 1) for i in range(18)]
    say("batch of 18")
    _batched(jobs, 11)
    o = ref.Oracle(base)
    for j in jobs[:3] + jobs[-2:]:
        want, _ = o.sart(j.p_host.astype(np.float32).astype(np.float64),
                         j.prior_host.astype(np.float32).astype(np.float64), 1, 0.5,
                         vox_weights=j.w_host.astype(np.float32).astype(np.float64))
        e = rel_l2(host(j.vol), want)
        say(j.name, "rel L2 vs oracle %.2e" % e)
        assert e <= 1.5e-6  # measured at most 1.1e-7


def test_batch_rejects_bad_items(torch_cuda):
    torch = torch_cuda
    from paper_2005_11976_amd import cyl
    j = _Job(torch, "tiny", I.config_tiny()["scan"], 1400, torch.float32, 1)
    e = j.entry()
    e.view = j.scan.n_views
    with pytest.raises(cyl.CylError) as ex:
        cyl.sart_batch_step([e])
    assert ex.value.code == cyl.CYL_EINVAL
    small = cyl.BatchEntry(j.G, 0, j.p, j.vol, j.ws[:16])
    with pytest.raises(cyl.CylError):
        cyl.sart_batch_step([small])
    j16 = _Job(torch, "tiny16", I.config_tiny()["scan"], 1401, torch.float16, 1)
    with pytest.raises(TypeError):
        cyl.sart_batch_step([j.entry(), j16.entry()])
    cyl.sart_batch_step([])
