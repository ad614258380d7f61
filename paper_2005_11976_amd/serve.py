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
    status: str = "done"  # "done", "cancelled" or "failed"
    error: str = ""


class Resident:
    """Class data kept on the device: prior volume and voxel weights."""

    def __init__(self, sc: I.ScanClass, dtype, device, phantom=None):
        import torch
        self.sc = sc
        ph = phantom if phantom is not None else I.industrial_phantom(sc.grid, sc.phantom_seed)
        self.prior = torch.from_numpy(ph.prior.astype(np.float32)).to(device).to(dtype).contiguous()
        self.weights = torch.from_numpy(ph.weights.astype(np.float32)).to(device).to(dtype).contiguous()
        self.nbytes = 2 * self.prior.numel() * self.prior.element_size()


def request_bytes(sc: I.ScanClass, itemsize):
    """Device bytes one admitted scan of class sc holds: projection difference
    (storage type) plus its FP32 staging, volume difference, result volume,
    the SART workspace (the FP32 residual image and its 8x8 tile maxima) and
    the geometry's device tables (its views, grid tables and FP dispatch
    orders, an upper bound)."""
    g = sc.grid
    rows, cols, nv = sc.det_rows, sc.det_cols, sc.views.shape[0]
    n_proj = nv * rows * cols
    tiles = ((rows + 7) // 8) * ((cols + 7) // 8)
    workspace = ((rows * cols + tiles) * 4 + 255) // 256 * 256
    geometry = nv * 256 + 24 * (g.n_r + g.n_h + g.n_theta + 3) + 3 * 4 * tiles + 4096
    return n_proj * (itemsize + 4) + 2 * g.n_vox * itemsize + workspace + geometry


def request_rays(sc: I.ScanClass):
    """Rays one SART step of a class-sc scan traces (one view)."""
    return sc.det_rows * sc.det_cols


class Scheduler:
    """Admission and stepping of a request stream, independent of the device.

    The executor does the work (`GpuExecutor` on the device; tests use a fake
    one on the CPU):
      now() -> seconds since the stream started; wait_until(t);
      admit(q, t) -> handle with .total sub-iterations (may raise: the request
        fails and frees what it took);
      step(handles) -> one sub-iteration for each (may raise: every scan of
        that step fails and is released, the others go on);
      finish(handle, rec) -> result of a completed scan; release(handle);
      drain() -> completion time of each record finished, once all work ended.
    Admission, in arrival order: when a slot is free (max_active), the scan's
    bytes (bytes_of(cls)) fit the budget next to the resident bytes, and the
    rays per step of the admitted scans stay within fill_rays (one scan is
    always admitted onto an idle executor).  A request whose bytes exceed what
    the budget leaves on an idle executor fails at once; the queue goes on.
    cancel: {rid: time}; a request cancelled before admission is dropped, an
    admitted one leaves at the first step boundary at or after that time.
    bypass: while the head of the queue waits only for ray capacity (a large
    scan behind running ones), up to this many later arrivals that fit are
    admitted past it, so that the GPU keeps work to overlap; then the head is
    waited for.
    """

    def __init__(self, bytes_of, rays_of, max_active=16, budget=64 << 30, resident_bytes=0,
                 fill_rays=327680, bypass=0):
        self.bytes_of, self.rays_of = bytes_of, rays_of
        self.max_active, self.budget, self.fill_rays = max_active, budget, fill_rays
        self.resident_bytes = resident_bytes
        self.bypass = bypass
        self.peak_active = 0
        self.bypassed = 0

    def run(self, requests, executor, cancel=None, progress=None):
        """progress(n): called with the number of records so far after each
        step that completes, cancels or fails a scan."""
        cancel = cancel or {}
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        active, records, results = [], [], {}
        used, rays = self.resident_bytes, 0
        head_rid, head_passed = None, 0

        def release(h):
            nonlocal used, rays
            used -= self.bytes_of(h.rec.cls)
            rays -= self.rays_of(h.rec.cls)
            executor.release(h)

        while pending or active:
            now = executor.now()
            # drop pending requests cancelled before their admission
            while pending and pending[0].rid in cancel and cancel[pending[0].rid] <= max(now, pending[0].arrival):
                q = pending.popleft()
                records.append(Record(q.rid, q.cls, q.arrival, status="cancelled"))
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                q = pending[0]
                need = self.bytes_of(q.cls)
                if used + need > self.budget:
                    if not active:
                        pending.popleft()
                        records.append(Record(q.rid, q.cls, q.arrival, status="failed",
                                              error="needs %d bytes, more than the budget leaves" % need))
                        continue
                    break
                if active and rays + self.rays_of(q.cls) > self.fill_rays:
                    # the head waits for ray capacity only: admit a later arrival that fits
                    if head_rid != q.rid:
                        head_rid, head_passed = q.rid, 0
                    if head_passed >= self.bypass:
                        break
                    pick = None
                    for i in range(1, len(pending)):
                        q2 = pending[i]
                        if q2.arrival > now:
                            break
                        if q2.rid in cancel and cancel[q2.rid] <= now:
                            continue
                        if (used + self.bytes_of(q2.cls) <= self.budget
                                and rays + self.rays_of(q2.cls) <= self.fill_rays):
                            pick = i
                            break
                    if pick is None:
                        break
                    q = pending[pick]
                    del pending[pick]
                    need = self.bytes_of(q.cls)
                    head_passed += 1
                    self.bypassed += 1
                else:
                    pending.popleft()
                rec = Record(q.rid, q.cls, q.arrival, admitted=now)
                try:
                    h = executor.admit(q, now)
                except Exception as e:  # noqa: BLE001 - the request fails, the stream goes on
                    rec.status, rec.error = "failed", str(e)
                    records.append(rec)
                    continue
                h.rec = rec
                used += need
                rays += self.rays_of(q.cls)
                active.append(h)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if pending:
                    executor.wait_until(pending[0].arrival)
                continue
            try:
                executor.step(active)
            except Exception as e:  # noqa: BLE001 - this step's scans fail, the stream goes on
                for h in active:
                    h.rec.status, h.rec.error = "failed", str(e)
                    records.append(h.rec)
                    release(h)
                active = []
                continue
            keep = []
            now = executor.now()
            for h in active:
                h.cursor += 1
                if h.cursor == h.total:
                    results[h.rec.rid] = executor.finish(h, h.rec)
                    records.append(h.rec)
                    release(h)
                elif h.rec.rid in cancel and cancel[h.rec.rid] <= now:
                    h.rec.status = "cancelled"
                    records.append(h.rec)
                    release(h)
                else:
                    keep.append(h)
            if progress and len(keep) < len(active):
                progress(len(records))
            active = keep
        executor.drain(records)
        records.sort(key=lambda r: r.rid)
        return records, results


class _Active:
    def __init__(self, geom, dproj, delta, ws, res, n_iter, lam):
        self.geom, self.dproj, self.delta, self.ws = geom, dproj, delta, ws
        self.res, self.cursor, self.lam = res, 0, lam
        self.total = n_iter * geom.scan.n_views
        self.rec = None

    def entry(self):
        return cyl.BatchEntry(self.geom, self.cursor % self.geom.scan.n_views, self.dproj, self.delta,
                              self.ws, vox_weights=self.res.weights, lam=self.lam)


class GpuExecutor:
    """Runs admitted scans on one GPU stream: one cyl_sart_batch_step per step
    (two kernel launches for up to 16 scans), at most two steps queued ahead of
    the GPU; times from CUDA events on that stream."""

    def __init__(self, residents, data, n_iter, lam, device, stream):
        import torch
        self.res, self.data, self.n_iter, self.lam = residents, data, n_iter, lam
        self.device, self.stream = device, stream
        self.dtype = residents[0].prior.dtype
        self.start = torch.cuda.Event(enable_timing=True)
        self.start.record(stream)
        self.t0 = time.perf_counter()
        self.inflight = collections.deque()
        self.retired = []   # geometries of released scans, destroyed once their last step is done
        self.done = {}      # rid -> completion event

    def now(self):
        return time.perf_counter() - self.t0

    def wait_until(self, t):
        wait = t - self.now()
        if wait > 0:
            time.sleep(wait)

    def admit(self, q, now):
        import torch
        r = self.res[q.cls]
        geom = cyl.Geometry(r.sc.scan(q.R, q.T), self.device)
        dev = "cuda:%d" % self.device
        p32 = torch.empty(geom.scan.proj_shape, dtype=torch.float32, device=dev)
        p32.copy_(self.data[q.rid], non_blocking=True)
        dproj = geom.fp_diff(r.prior, p32, out_dtype=self.dtype, stream=self.stream)
        del p32  # stream-ordered: its memory is reused only by later work on this stream
        delta = torch.zeros_like(r.prior)
        ws = torch.empty(geom.workspace_bytes(), dtype=torch.uint8, device=dev)
        return _Active(geom, dproj, delta, ws, r, self.n_iter, self.lam)

    def step(self, handles):
        import torch
        cyl.sart_batch_step([h.entry() for h in handles], self.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        self.inflight.append(ev)
        if len(self.inflight) > 2:
            self.inflight.popleft().synchronize()
        while self.retired and self.retired[0][1].query():
            self.retired.pop(0)[0].close()

    def finish(self, h, rec):
        import torch
        vol = cyl.add(h.res.prior, h.delta, stream=self.stream)
        done = torch.cuda.Event(enable_timing=True)
        done.record(self.stream)
        self.done[rec.rid] = done
        return vol

    def release(self, h):
        import torch
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.retired.append((h.geom, ev))

    def drain(self, records):
        self.stream.synchronize()
        for g, _ in self.retired:
            g.close()
        self.retired = []
        for rec in records:
            if rec.rid in self.done:
                rec.finished = self.start.elapsed_time(self.done[rec.rid]) * 1e-3
                rec.latency = rec.finished - rec.arrival


class Server:
    """Continuous batching of SART scans on one GPU (see module docstring).

    max_active: batch slots (scans stepped together; 16 fill one launch pair).
    hbm_budget: bytes for resident class data plus admitted scans.
    fill_rays: rays per step above which no further scan joins (one 512x512
      view fills the GPU); a scan is always admitted onto an idle GPU.
    """

    def __init__(self, residents, n_iter=15, lam=0.5, max_active=16, hbm_budget=64 << 30,
                 fill_rays=327680, device=0, stream=None, bypass=4):
        import torch
        self.bypass = bypass
        self.res = residents
        self.n_iter, self.lam = n_iter, lam
        self.max_active, self.budget, self.fill_rays = max_active, hbm_budget, fill_rays
        self.device = device
        self.stream = stream or torch.cuda.Stream(device=device)
        self.dtype = residents[0].prior.dtype
        self.resident_bytes = sum(r.nbytes for r in residents)
        if self.resident_bytes > hbm_budget:
            raise ValueError("resident class data exceeds the HBM budget")
        self.peak_active = 0

    def run(self, requests, data, cancel=None, progress=None):
        """Serve `requests` (inputs.Request, arrival seconds from now) whose
        projections are data[rid] (pinned host tensors, FP32).  Returns
        (records, volumes): per-request timing and status, and the result
        volume of every scan that completed.  progress: see Scheduler.run."""
        import torch
        itemsize = torch.empty((), dtype=self.dtype).element_size()
        sched = Scheduler(lambda c: request_bytes(self.res[c].sc, itemsize),
                          lambda c: request_rays(self.res[c].sc), self.max_active, self.budget,
                          self.resident_bytes, self.fill_rays, self.bypass)
        with torch.cuda.stream(self.stream):
            ex = GpuExecutor(self.res, data, self.n_iter, self.lam, self.device, self.stream)
            records, volumes = sched.run(requests, ex, cancel, progress)
        self.peak_active = sched.peak_active
        self.bypassed = sched.bypassed
        for rec in records:
            if rec.status == "failed" and "budget" in rec.error:
                raise ValueError("request %d %s" % (rec.rid, rec.error))
        return records, volumes


def run_fifo(residents, requests, data, n_iter=15, lam=0.5, device=0, stream=None, progress=None):
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
            if progress:
                progress(len(finished))
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
