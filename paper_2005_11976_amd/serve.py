"""Continuous-batching SART server for a stream of scans (in-line inspection).

Requests arrive over time; each is a scan of one of a few object classes (grid,
trajectory, detector) with its own pose and its measured FP32 projections (in
pinned host memory when it arrives).  The server keeps each class's prior
volume and voxel weights resident on the device (the prior of Sec. 2.2 is per
part type), and runs weighted SART (Eq. 7, one projection per update) for every
admitted scan, in low-precision storage:

  * difference form: SART from the prior mu0 on data p equals mu0 + SART from 0
    on d = p - A mu0 (Eq. 7 is affine in mu and p).  The server stores d and the
    volume difference delta in the storage type (FP16 by default); both are
    small where the prior is right, so their rounding costs far less than
    rounding mu and p themselves.  d is formed in FP32 on the device
    (cyl_fp_diff), the result mu0 + delta by cyl_add;
  * admission: in arrival order, when a batch slot is free, the scan's device
    memory fits the HBM budget next to the resident class data, and the rays
    per step of the admitted scans stay within a fill cap (one large scan
    already fills the GPU, so large scans run nearly alone and small ones are
    packed together);
  * stepping: every step runs one SART sub-iteration for every admitted scan in
    one batched call (cyl_sart_batch_step: two kernel launches for up to 16
    scans), so scans that arrive while others run join the next step and
    share its launches; a scan leaves after its last sub-iteration;
  * latency: from arrival to the GPU completion of the scan's result.

The result of a scan does not depend on which other scans share its steps
(the kernels treat batch items independently); the GPU tests check this bit
for bit.  All device arithmetic runs in the HIP kernels of libcyl; this module
only schedules calls.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import cyl
from . import inputs as I


@dataclasses.dataclass
class Record:
    rid: int
    cls: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    latency: float = 0.0


class Resident:
    """Class data kept on the device: prior volume and voxel weights."""

    def __init__(self, sc: I.ScanClass, dtype, device, phantom=None):
        import torch
        self.sc = sc
        ph = phantom if phantom is not None else I.industrial_phantom(sc.grid, sc.phantom_seed)
        self.prior = torch.from_numpy(ph.prior.astype(np.float32)).to(device).to(dtype).contiguous()
        self.weights = torch.from_numpy(ph.weights.astype(np.float32)).to(device).to(dtype).contiguous()
        self.nbytes = 2 * self.prior.numel() * self.prior.element_size()


class _Active:
    def __init__(self, rec, geom, dproj, delta, ws, res, n_iter, lam):
        self.rec, self.geom, self.dproj, self.delta, self.ws = rec, geom, dproj, delta, ws
        self.res, self.cursor, self.lam = res, 0, lam
        self.total = n_iter * geom.scan.n_views

    def entry(self):
        return cyl.BatchEntry(self.geom, self.cursor % self.geom.scan.n_views, self.dproj, self.delta,
                              self.ws, vox_weights=self.res.weights, lam=self.lam)


def request_bytes(sc: I.ScanClass, itemsize):
    """Device bytes one admitted scan of class sc holds: projection difference
    (storage type) plus its FP32 staging, volume difference, result volume and
    the FP32 residual image."""
    g = sc.grid
    n_proj = sc.views.shape[0] * sc.det_rows * sc.det_cols
    return (n_proj * (itemsize + 4) + 2 * g.n_vox * itemsize
            + ((sc.det_rows * sc.det_cols * 4 + 255) // 256) * 256)


def request_rays(sc: I.ScanClass):
    """Rays one SART step of a class-sc scan traces (one view)."""
    return sc.det_rows * sc.det_cols


class Server:
    """Continuous batching of SART scans on one GPU (see module docstring).

    max_active: batch slots (scans stepped together; 16 fill one launch pair).
    hbm_budget: bytes for resident class data plus admitted scans.
    fill_rays: rays per step above which no further scan joins (one 512x512
      view fills the GPU); a scan is always admitted onto an idle GPU.
    """

    def __init__(self, residents, n_iter=15, lam=0.5, max_active=16, hbm_budget=64 << 30,
                 fill_rays=327680, device=0, stream=None):
        import torch
        self.res = residents
        self.n_iter, self.lam = n_iter, lam
        self.max_active, self.budget, self.fill_rays = max_active, hbm_budget, fill_rays
        self.device = device
        self.stream = stream or torch.cuda.Stream(device=device)
        self.dtype = residents[0].prior.dtype
        self.resident_bytes = sum(r.nbytes for r in residents)
        if self.resident_bytes > hbm_budget:
            raise ValueError("resident class data exceeds the HBM budget")

    def run(self, requests, data):
        """Serve `requests` (inputs.Request, arrival seconds from now) whose
        projections are data[rid] (pinned host tensors in the storage dtype).
        Returns (records, volumes): per-request timing and result volumes."""
        import torch
        itemsize = torch.empty((), dtype=self.dtype).element_size()
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        active, finished, volumes = [], [], {}
        retired = []  # geometries of finished scans, destroyed once their last step is done
        used = self.resident_bytes
        rays = 0
        inflight = collections.deque()
        start = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(self.stream):
            start.record(self.stream)
            t0 = time.perf_counter()
            while pending or active:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now and len(active) < self.max_active:
                    q = pending[0]
                    sc = self.res[q.cls].sc
                    need = request_bytes(sc, itemsize)
                    if used + need > self.budget:
                        if not active:
                            raise ValueError("request %d needs %d bytes, more than the HBM budget "
                                             "leaves" % (q.rid, need))
                        break
                    if active and rays + request_rays(sc) > self.fill_rays:
                        break
                    pending.popleft()
                    used += need
                    rays += request_rays(sc)
                    active.append(self._admit(q, data[q.rid], now))
                if not active:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                    continue
                cyl.sart_batch_step([a.entry() for a in active], self.stream)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.stream)
                keep = []
                for a in active:
                    a.cursor += 1
                    if a.cursor == a.total:
                        volumes[a.rec.rid] = cyl.add(a.res.prior, a.delta, stream=self.stream)
                        done = torch.cuda.Event(enable_timing=True)
                        done.record(self.stream)
                        finished.append((a.rec, done))
                        used -= request_bytes(a.res.sc, itemsize)
                        rays -= request_rays(a.res.sc)
                        retired.append((a.geom, done))
                    else:
                        keep.append(a)
                active = keep
                # keep at most two steps queued ahead of the GPU
                inflight.append(ev)
                if len(inflight) > 2:
                    inflight.popleft().synchronize()
                while retired and retired[0][1].query():
                    retired.pop(0)[0].close()
            self.stream.synchronize()
            for g, _ in retired:
                g.close()
        records = []
        for rec, ev in finished:
            rec.finished = start.elapsed_time(ev) * 1e-3
            rec.latency = rec.finished - rec.arrival
            records.append(rec)
        records.sort(key=lambda r: r.rid)
        return records, volumes

    def _admit(self, q, host_proj, now):
        import torch
        r = self.res[q.cls]
        geom = cyl.Geometry(r.sc.scan(q.R, q.T), self.device)
        dev = "cuda:%d" % self.device
        p32 = torch.empty(geom.scan.proj_shape, dtype=torch.float32, device=dev)
        p32.copy_(host_proj, non_blocking=True)
        dproj = geom.fp_diff(r.prior, p32, out_dtype=self.dtype, stream=self.stream)
        del p32  # stream-ordered: its memory is reused only by later work on this stream
        delta = torch.zeros_like(r.prior)
        ws = torch.empty(geom.workspace_bytes(), dtype=torch.uint8, device=dev)
        return _Active(Record(q.rid, q.cls, q.arrival, admitted=now), geom, dproj, delta, ws, r,
                       self.n_iter, self.lam)


def run_fifo(residents, requests, data, n_iter=15, lam=0.5, device=0, stream=None):
    """The plain per-scan loop: requests in arrival order, one cyl_sart_run
    each on its own (no batching), queued on one stream as they arrive; same
    timing rules as Server.run."""
    import torch
    stream = stream or torch.cuda.Stream(device=device)
    finished, volumes, geoms = [], {}, []
    start = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        t0 = time.perf_counter()
        for q in sorted(requests, key=lambda x: x.arrival):
            r = residents[q.cls]
            wait = q.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            geom = cyl.Geometry(r.sc.scan(q.R, q.T), device)
            geoms.append(geom)  # destroyed after the stream has drained
            proj = torch.empty(geom.scan.proj_shape, dtype=r.prior.dtype, device="cuda:%d" % device)
            proj.copy_(data[q.rid], non_blocking=True)  # FP32 data, FP32 prior: the plain loop
            vol = r.prior.clone()
            geom.sart(proj, vol, n_iter, lam, vox_weights=r.weights, stream=stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            finished.append((Record(q.rid, q.cls, q.arrival), ev))
            volumes[q.rid] = vol
        stream.synchronize()
    for g in geoms:
        g.close()
    records = []
    for rec, ev in finished:
        rec.finished = start.elapsed_time(ev) * 1e-3
        rec.latency = rec.finished - rec.arrival
        records.append(rec)
    records.sort(key=lambda r: r.rid)
    return records, volumes


def latency_summary(records):
    lat = np.array([r.latency for r in records])
    span = max(r.finished for r in records) - min(r.arrival for r in records)
    return {"requests": len(records), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "makespan_s": float(span), "scans_per_s": len(records) / span}


def make_request_data(residents, requests, device=0, phantoms=None):
    """Measured FP32 projections of each request (synthetic: the GPU forward
    projection of its class phantom under its pose), in pinned host memory."""
    import torch
    out = {}
    truths = {}
    for q in requests:
        r = residents[q.cls]
        if q.cls not in truths:
            ph = phantoms[q.cls] if phantoms else I.industrial_phantom(r.sc.grid, r.sc.phantom_seed)
            truths[q.cls] = torch.from_numpy(ph.truth.astype(np.float32)).to(device)
        g = cyl.Geometry(r.sc.scan(q.R, q.T), device)
        p = g.fp(truths[q.cls])
        out[q.rid] = p.cpu().pin_memory()
        g.close()
    return out
