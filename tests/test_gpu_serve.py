"""The continuous-batching server: each scan's result is the same alone and in
the mix (bitwise), admission respects slots and the HBM budget, and the FP16
served results (difference form: prior + delta, both FP16) stay within 1e-3
relative L2 of the plain per-scan FP32 loop: the rounding of the resident prior
and of the result are each at most u = 2^-11 relative, and the stored
differences are small."""
import numpy as np
import pytest

from paper_2005_11976_amd import inputs as I
from tests.gpu_util import host, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_11976_amd import cyl, serve
    cyl.lib()
    classes = [
        I.ScanClass("a", I.Grid(16, 64, 16, 0.0, 10.0, -5.0, 5.0), I.circular_views(8, 100.0, 200.0, 0.4),
                    32, 48, 1060),
        I.ScanClass("b", I.Grid(24, 72, 12, 0.0, 25.0, -25.0, 25.0), I.circular_views(11, 200.0, 400.0, 1.6),
                    40, 36, 1061),
    ]
    phantoms = [I.industrial_phantom(c.grid, c.phantom_seed, n_annuli=3, n_incl=3) for c in classes]
    reqs = [I.Request(q.rid, q.cls, q.arrival, q.R, q.T) for q in I.serving_requests(7, 200.0, n_classes=2)]
    res16 = [serve.Resident(c, torch.float16, 0, ph) for c, ph in zip(classes, phantoms)]
    res32 = [serve.Resident(c, torch.float32, 0, ph) for c, ph in zip(classes, phantoms)]
    data = serve.make_request_data(res32, reqs, phantoms=phantoms)
    return torch, serve, classes, reqs, res16, res32, data


def test_served_equals_alone_and_fifo(setup):
    torch, serve, classes, reqs, res16, res32, data = setup
    n_iter = 2
    say("serve mixed", len(reqs), "requests")
    srv = serve.Server(res16, n_iter=n_iter, max_active=4)
    recs, vols = srv.run(reqs, data)
    assert len(recs) == len(reqs) and all(r.latency > 0 and r.status == "done" for r in recs)
    say("serve", serve.latency_summary(recs), "peak active scans", srv.peak_active)
    assert srv.peak_active > 1  # the burst of arrivals shares steps
    say("fifo fp32")
    frecs, fvols = serve.run_fifo(res32, reqs, data, n_iter=n_iter)
    for q in reqs:
        say("alone", q.rid)
        alone = serve.Server(res16, n_iter=n_iter, max_active=1)
        r1, v1 = alone.run([I.Request(q.rid, q.cls, 0.0, q.R, q.T)], data)
        assert torch.equal(v1[q.rid], vols[q.rid]), q.rid
        sc = classes[q.cls]
        e = rel_l2(host(vols[q.rid]), host(fvols[q.rid]))
        say("request", q.rid, "class", sc.name, "fp16 served vs fp32 per-scan rel L2 %.2e" % e)
        assert e <= 1e-3


def test_budget_limits_admission(setup):
    torch, serve, classes, reqs, res16, res32, data = setup
    from paper_2005_11976_amd.serve import request_bytes
    one = max(request_bytes(c, 2) for c in classes)
    srv = serve.Server(res16, n_iter=1, max_active=16, hbm_budget=srv_res_bytes(res16) + one)
    say("serve with a budget of one scan")
    recs, vols = srv.run(reqs, data)
    assert srv.peak_active == 1
    ref = serve.Server(res16, n_iter=1, max_active=16)
    recs2, vols2 = ref.run(reqs, data)
    for q in reqs:
        assert torch.equal(vols[q.rid], vols2[q.rid])
    # one scan at a time: every admission after the previous scan's last step was enqueued
    adm = sorted(r.admitted for r in recs)
    assert len(adm) == len(reqs)
    with pytest.raises(ValueError):
        serve.Server(res16, n_iter=1, hbm_budget=srv_res_bytes(res16) + 16).run(reqs[:1], data)


def srv_res_bytes(res):
    return sum(r.nbytes for r in res)
