"""Benchmark: weighted SART on the 256 x 720 x 128 cylindrical grid (one GPU).

One step = one SART iteration: for each of the 120 views, the forward
projection with the residual epilogue and the back-projection with the
weighted update epilogue (all hot-path kernels), on a synthetic industrial
part (6 coaxial annuli, 8 ring-sector inclusions, one missing), starting from
the prior, voxel weights 1 in the inclusion ring and 0.25 elsewhere.

Prints one JSON line with SART iterations/s, Grays/s (fwd+bp), the roofline
of the dominant kernel (HIP-event kernel times) and the FP64 oracle timed on
the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch (read + written) of the FP32 SART kernels on this
# workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE passes scaled by a 1 GiB
# device copy, taken on the kernel sources whose sha256 prefix is given here
# (profiles/fp_bp_sart_single_256x720x128_hbm_counters.md). For any other
# source, or another storage type, the traffic is reported as null.
MEASURED_TRAFFIC = {"src_sha": "be1e93b74c6bdafc",
                    "fp_residual": 143590000 + 1210163,
                    "bp_update": 193154000 + 93194035}
# VALU wave-instructions per launch (rocprofv3 SQ_INSTS_VALU) of the same
# sources (profiles/fp_bp_sart_single_256x720x128_valu_counters.md).  A wave64
# VALU instruction takes 4 cycles of a 16-lane SIMD (packed FP32 is off), so
# the issue capacity of a launch is 1024 SIMDs x 2.4 GHz x duration / 4.
# active_lanes: SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU), the fraction of
# the 64 lanes that work in an average VALU instruction.
MEASURED_VALU = {"src_sha": "be1e93b74c6bdafc", "fp_residual": 1.018e8, "bp_update": 2.311e8,
                 "active_lanes": {"fp_residual": 0.951, "bp_update": 0.696}}
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("cyl_kernels.hip", "cyl_host.cpp", "cyl_internal.h", "cyl_ray.h", "cyl_block.h", "cyl_isa.h",
              "cyl_store.h"):
        with open(os.path.join(ROOT, "paper_2005_11976_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP16/BF16 storage measurement")
    ap.add_argument("--kernel-views", type=int, default=120,
                    help="views in the per-kernel HIP-event timing pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests in the serving measurement (0 = skip it)")
    ap.add_argument("--serve-iters", type=int, default=15)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, scans/s")
    ap.add_argument("--core-only", action="store_true",
                    help="only the SART sweep and the per-kernel timing (for profiler runs: the ordered-subset, "
                         "pose and serving parts launch the same kernels with other shapes)")
    return ap.parse_args()


def serving(args):
    """Continuous batching (FP16 storage) against the plain per-scan FP32 loop
    on the same request stream: classes A/B/C, seeded poses, Poisson arrivals."""
    import torch
    from paper_2005_11976_amd import inputs as I, serve
    classes = I.serving_classes()
    reqs = I.serving_requests(args.serve_requests, args.serve_rate)
    used = sorted({q.cls for q in reqs})
    log("serving:", len(reqs), "requests, classes", [classes[c].name for c in used])
    phantoms = [I.industrial_phantom(c.grid, c.phantom_seed) for c in classes]
    res16 = [serve.Resident(c, torch.float16, 0, ph) for c, ph in zip(classes, phantoms)]
    res32 = [serve.Resident(c, torch.float32, 0, ph) for c, ph in zip(classes, phantoms)]
    data = serve.make_request_data(res32, reqs, phantoms=phantoms)  # measured FP32 projections
    del phantoms
    torch.cuda.synchronize()
    srv = serve.Server(res16, n_iter=args.serve_iters, max_active=16, hbm_budget=64 << 30)
    log("serving: batched run")
    def prog(n):
        if n % 16 == 0:
            log("serving: %d of %d requests done" % (n, len(reqs)))
    recs, vols = srv.run(reqs, data, progress=prog)
    log("serving: per-scan FP32 run")
    frecs, fvols = serve.run_fifo(res32, reqs, data, n_iter=args.serve_iters, progress=prog)
    errs = [float((vols[q.rid].float() - fvols[q.rid]).norm() / fvols[q.rid].norm()) for q in reqs]
    b, f = serve.latency_summary(recs), serve.latency_summary(frecs)
    log("serving: batched p50 %.2f s p99 %.2f s %.3f scans/s; fifo p50 %.2f s p99 %.2f s %.3f scans/s"
        % (b["p50_s"], b["p99_s"], b["scans_per_s"], f["p50_s"], f["p99_s"], f["scans_per_s"]))
    return {"requests": len(reqs), "rate_per_s": args.serve_rate, "iterations": args.serve_iters,
            "classes": "".join(classes[c].name for c in used),
            "dtype": "f16 storage (prior + difference form), f32 arithmetic",
            "hbm_budget_gb": 64, "slots": 16, "fill_rays": srv.fill_rays, "bypass": srv.bypass,
            "bypassed_admissions": srv.bypassed, "peak_active_scans": srv.peak_active,
            "batched": b, "per_scan_fp32": f,
            "throughput_ratio": b["scans_per_s"] / f["scans_per_s"],
            "p99_ratio": b["p99_s"] / f["p99_s"],
            "rel_err_vs_per_scan_fp32": {"max": max(errs), "mean": float(np.mean(errs))}}


def projector_rates(G, scan, truth, p):
    """FP-only and BP-only rates: cyl_fp and cyl_bp over all views of the scan
    (one call each; HIP-event time, median of 3 after a warm-up), as Grays/s
    (each detector pixel of each view counts once)."""
    import torch
    proj = torch.empty_like(p)
    vol = torch.empty_like(truth)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    fp_ms = timed(lambda: G.fp(truth, proj))
    bp_ms = timed(lambda: G.bp(p, vol))
    rays = scan.n_views * scan.det_rows * scan.det_cols
    log("projectors over %d views: fp %.2f ms (%.2f Grays/s), bp %.2f ms (%.2f Grays/s)"
        % (scan.n_views, fp_ms, rays / fp_ms / 1e6, bp_ms, rays / bp_ms / 1e6))
    return {"views": scan.n_views, "fp_ms": fp_ms, "fp_grays_per_s": rays / fp_ms / 1e6,
            "bp_ms": bp_ms, "bp_grays_per_s": rays / bp_ms / 1e6}


def posed_large():
    """Weighted SART from the prior on the 512x1440x256 posed scan (60 views of
    1024 x 768, seeded pose, Poisson data at 1e4 photons): one warm-up and two
    timed iterations (HIP events), with the error against the truth."""
    import torch
    from paper_2005_11976_amd import cyl, inputs as I
    cfg = I.config_posed()
    scan = cfg["scan"]
    log("posed large: phantom and data", scan.grid.shape, scan.proj_shape)
    ph = I.industrial_phantom(scan.grid, cfg["seed"])
    G = cyl.Geometry(scan, 0)
    truth = torch.from_numpy(ph.truth.astype(np.float32)).cuda()
    clean = G.fp(truth).cpu().numpy()
    p = torch.from_numpy(I.poisson_line_integrals(clean, cfg["photons"], cfg["noise_seed"]).astype(np.float32)).cuda()
    prior = torch.from_numpy(ph.prior.astype(np.float32)).cuda()
    w = torch.from_numpy(ph.weights.astype(np.float32)).cuda()
    ws = torch.empty(G.workspace_bytes(), dtype=torch.uint8, device="cuda")
    vol = prior.clone()
    G.sart(p, vol, 1, cfg["lam"], vox_weights=w, workspace=ws)
    torch.cuda.synchronize()
    n = 2
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    G.sart(p, vol, 1 + n, cfg["lam"], vox_weights=w, workspace=ws, start_iter=1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    err = float((vol - truth).norm() / truth.norm())
    G.close()
    log("posed large: %.3f SART it/s (%.2f ms per view), error vs truth %.4f after %d iterations"
        % (1000.0 / ms, ms / scan.n_views, err, 1 + n))
    return {"workload": cfg["name"], "grid": list(scan.grid.shape), "views": scan.n_views,
            "detector": [scan.det_rows, scan.det_cols], "it_per_s": 1000.0 / ms, "ms_per_view": ms / scan.n_views,
            "iterations_timed": n, "rel_err_vs_truth": err, "data": "synthetic, Poisson at 1e4 photons"}


def pose_estimation(scan):
    """Sec. 2.1 on the 256x720x128 scan geometry: a solid cylinder (r <= 20 mm,
    |h| <= 20 mm: one symmetric feature, as the paper segments) posed with a
    seeded tilt and shift, its 120 projections from cyl_fp, the corner kernel
    (HIP-event time per call, mean of 20 back-to-back calls), host point tracking of the two axis points, and the axis
    error against the known pose (the internal rotation is not estimated)."""
    import math
    import torch
    from paper_2005_11976_amd import cyl, inputs as I
    g = scan.grid
    dh, dr = (g.h_max - g.h_min) / g.n_h, (g.r_max - g.r_min) / g.n_r
    vol = torch.zeros(g.shape, dtype=torch.float32)
    vol[int(round((-20.0 - g.h_min) / dh)):int(round((20.0 - g.h_min) / dh)), :, :int(round(20.0 / dr))] = 0.02
    R, T, prm = I.random_pose(2002)
    posed = I.Scan(g, scan.views, scan.det_rows, scan.det_cols, R, T)
    G = cyl.Geometry(posed, 0)
    p = G.fp(vol.cuda())
    thr = float(np.float32(0.02))
    cyl.axis_corners(p, thr, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20  # back-to-back calls: the host's per-call binding time overlaps the kernels
    e0.record()
    for _ in range(reps):
        corners = cyl.axis_corners(p, thr, 1)
    e1.record()
    torch.cuda.synchronize()
    kernel_ms = e0.elapsed_time(e1) / reps
    t0 = time.perf_counter()
    top_uv, bot_uv, valid = cyl.axis_points(corners.cpu().numpy())
    a, _ = cyl.track_point(posed.views, posed.det_rows, posed.det_cols, top_uv, valid)
    b, _ = cyl.track_point(posed.views, posed.det_rows, posed.det_cols, bot_uv, valid)
    host_ms = (time.perf_counter() - t0) * 1e3
    d = (b - a) / np.linalg.norm(b - a)
    d_true = R.T @ np.array([0.0, 0.0, 1.0])
    ang = math.degrees(math.acos(min(1.0, abs(float(d @ d_true)))))
    c_true = -R.T @ T
    mid = 0.5 * (a + b)
    off = (mid - c_true) - ((mid - c_true) @ d_true) * d_true
    G.close()
    log("pose: corners %.3f ms (120 views), tracking %.2f ms, axis error %.3f deg, %.3f mm"
        % (kernel_ms, host_ms, ang, float(np.linalg.norm(off))))
    return {"views": scan.n_views, "detector": [scan.det_rows, scan.det_cols], "corner_kernel_ms": kernel_ms,
            "tracking_host_ms": host_ms, "axis_error_deg": ang, "axis_offset_mm": float(np.linalg.norm(off)),
            "true_tilt_deg": math.degrees(prm["beta"])}


def ordered_subsets(G, scan, p, prior, w, lam, truth):
    """Eq. 7 with ordered subsets of several projections on the same scan
    (cyl_os_sart_run): iterations/s and the distance to the truth after as
    for one view per update (the paper's SART, for reference), 10 views per
    update, and SIRT (all 120), 3 iterations each from the prior."""
    import torch
    out = {}
    for m in (1, 10, scan.n_views):
        ws = torch.empty(G.os_workspace_bytes(m), dtype=torch.uint8, device="cuda")
        vol = prior.clone()
        G.os_sart(p, vol, 1, m, lam, vox_weights=w, workspace=ws)  # warm-up
        vol.copy_(prior)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = 3
        e0.record()
        G.os_sart(p, vol, n, m, lam, vox_weights=w, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        rel = float((vol.float() - truth).norm() / truth.norm())
        key = "sirt" if m == scan.n_views else ("sart" if m == 1 else "os%d" % m)
        out[key] = {"views_per_update": m, "it_per_s": 1000.0 / ms, "ms_per_iter": ms, "iterations": n,
                    "rel_err_vs_truth": rel}
        log("ordered subsets of %d views: %.2f it/s, rel err vs truth after %d it %.4f" % (m, 1000.0 / ms, n, rel))
        del ws
    return out


def comparison_projectors(G, scan, p, prior, w, lam, truth, nv=8):
    """The paper's own pair (Sec. 2.2) beside the exact one on the same scan:
    per-view times of the sampled FP (nearest and trilinear, step = half the
    radial cell) and of the voxel-driven BP against the exact FP and BP, the
    sampled projections' distance from the exact line integrals of the
    truth, and 3 SART iterations with the pair from the prior (error against
    the truth beside the exact pair's)."""
    import torch
    g = scan.grid
    step = 0.5 * (g.r_max - g.r_min) / g.n_r
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps / nv

    exact = p[:nv].float()
    out = {"step_mm": step, "views_timed": nv}
    buf = torch.empty_like(p)
    out["exact_fp_ms_per_view"] = timed(lambda: G.fp(truth, buf, 0, nv))
    for interp, name in ((0, "nearest"), (1, "linear")):
        out["sampled_fp_%s_ms_per_view" % name] = timed(lambda: G.fp_sampled(truth, step, interp, buf, 0, nv))
        q = buf[:nv].float()
        out["sampled_fp_%s_rel_err_vs_exact" % name] = float((q - exact).norm() / exact.norm())
    vol = torch.empty_like(truth)
    out["exact_bp_ms_per_view"] = timed(lambda: G.bp(p, vol, 0, nv))
    out["voxel_bp_ms_per_view"] = timed(lambda: G.bp_voxel(p, vol, 0, nv))
    v = prior.clone()
    G.sart_sampled(p, v, 1, step, 1, lam, vox_weights=w)  # warm-up
    v.copy_(prior)
    torch.cuda.synchronize()
    ev[0].record()
    G.sart_sampled(p, v, 3, step, 1, lam, vox_weights=w)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 3
    out["sampled_sart_linear"] = {"it_per_s": 1000.0 / ms, "iterations": 3,
                                  "rel_err_vs_truth": float((v.float() - truth).norm() / truth.norm())}
    log("paper's pair: sampled FP %.3f / %.3f ms per view (nearest / linear; exact %.3f), rel err vs exact "
        "%.2e / %.2e; voxel BP %.3f ms (exact %.3f); SART %.2f it/s, err vs truth %.4f"
        % (out["sampled_fp_nearest_ms_per_view"], out["sampled_fp_linear_ms_per_view"], out["exact_fp_ms_per_view"],
           out["sampled_fp_nearest_rel_err_vs_exact"], out["sampled_fp_linear_rel_err_vs_exact"],
           out["voxel_bp_ms_per_view"], out["exact_bp_ms_per_view"], out["sampled_sart_linear"]["it_per_s"],
           out["sampled_sart_linear"]["rel_err_vs_truth"]))
    return out


def symmetric_matrix(G, scan, p, prior, w, lam, truth):
    """The reuse of view 0's exact system matrix for every view of this
    unposed scan (cyl_sym_*, the acceleration the posed method gives up):
    build time, entries, device bytes, SART iterations/s over 3 iterations
    from the prior and the distance to the truth (the same arithmetic as the
    traversal path, summed in another order)."""
    import torch
    from paper_2005_11976_amd import cyl
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = cyl.SymMatrix(G)
    build_s = time.perf_counter() - t0
    v = prior.clone()
    S.sart(p, v, 1, lam, vox_weights=w)  # warm-up
    v.copy_(prior)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.sart(p, v, 3, lam, vox_weights=w)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    nnz = S.nnz
    out = {"build_s": build_s, "nnz_per_view": nnz,
           "device_bytes": nnz * 18 + scan.grid.n_vox * 8 + scan.det_rows * scan.det_cols * 8,
           "sart_it_per_s": 1000.0 / ms, "ms_per_view": ms / scan.n_views, "iterations": 3,
           "rel_err_vs_truth": float((v.float() - truth).norm() / truth.norm())}
    log("symmetric matrix: build %.2f s, %d entries, SART %.2f it/s (%.3f ms per view), err vs truth %.4f"
        % (build_s, nnz, out["sart_it_per_s"], out["ms_per_view"], out["rel_err_vs_truth"]))
    S.close()
    return out


def cpu_info():
    """Host CPU model and core counts (for the CPU baseline's record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(scan, truth, prior, weights, p, nthreads):
    """The FP64 oracle (test infrastructure) on a bounded sample: one SART
    sub-iteration (FP + residual + BP + update) for 8 of the 120 views
    (k = 0, 15, ..., 105; about 15 s on 16 host threads), scaled to SART
    iterations/s."""
    from oracle import ref
    o = ref.Oracle(scan)
    sample_views = list(range(0, 120, 15))
    t0 = time.perf_counter()
    P = scan.det_rows * scan.det_cols
    mu = prior.astype(np.float64).ravel().copy()
    w = weights.astype(np.float64).ravel()
    for k in sample_views:
        q, L = o.fp(mu, k, k + 1, nthreads=nthreads, rowsum=True)
        res = p[k].astype(np.float64) - q[0]
        rho = np.where(L[0] > 0, res / np.where(L[0] > 0, L[0], 1.0), 0.0)
        c, n = o.bp(rho, k, k + 1, nthreads=nthreads, colsum=True)
        c, n = c.ravel(), n.ravel()
        upd = np.where(n > 0, 0.5 * w * c / np.where(n > 0, n, 1.0), 0.0)
        mu += upd
    dt = time.perf_counter() - t0
    per_view = dt / len(sample_views)
    it_s = 1.0 / (per_view * scan.n_views)
    out = {"value": it_s, "unit": "SART it/s", "cores": nthreads, "kind": "oracle",
           "sample": "%d of %d views (k = 0, 15, ..., 105; one SART sub-iteration each, %.1f s), scaled x%d"
                     % (len(sample_views), scan.n_views, dt, scan.n_views / len(sample_views)),
           "seconds": dt,
           "threads_note": "the oracle's own threads, capped at the 16 host threads a one-GPU job is given"}
    out.update(cpu_info())
    return out


def mixed_precision(cfg, ph, p32, nthreads, steps=3):
    """FP16 and BF16 storage (Eq. 7 with the volume, data and weights stored in
    16 bits, FP32 arithmetic): SART it/s on the full 256x720x128 scan, and the
    relative L2 distance to the FP64 oracle's iterates after each of 2
    iterations over 12 of its views (every 10th), from the same prior and on
    the same data (the FP32 projections the bench measures with), FP32
    alongside."""
    import torch
    from oracle import ref
    from paper_2005_11976_amd import cyl, inputs as I
    scan = cfg["scan"]
    lam = cfg["lam"]
    out = {}
    # rates on the full scan
    G = cyl.Geometry(scan, 0)
    ws = torch.empty(G.workspace_bytes(), dtype=torch.uint8, device="cuda")
    for name, tdt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        p = p32.to(tdt).contiguous()
        prior = torch.from_numpy(ph.prior.astype(np.float32)).cuda().to(tdt).contiguous()
        w = torch.from_numpy(ph.weights.astype(np.float32)).cuda().to(tdt).contiguous()
        vol = prior.clone()
        G.sart(p, vol, 1, lam, vox_weights=w, workspace=ws)
        vol.copy_(prior)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for s in range(steps):
            G.sart(p, vol, s + 1, lam, vox_weights=w, workspace=ws, start_iter=s)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"value": 1000.0 * steps / e0.elapsed_time(e1), "unit": "SART it/s"}
        log("mixed %s: %.3f SART it/s" % (name, out[name]["value"]))
    del ws
    # accuracy against the FP64 oracle on 12 views
    sub = I.Scan(scan.grid, scan.views[::10], scan.det_rows, scan.det_cols, scan.R, scan.T)
    data = p32[::10].contiguous()
    data64 = data.cpu().numpy().astype(np.float64)
    wts = ph.weights.astype(np.float32)
    mu = ph.prior.astype(np.float32).astype(np.float64)
    ref_iters = []
    t0 = time.perf_counter()
    for it in range(2):
        for k in range(sub.n_views):
            one = I.Scan(sub.grid, sub.views[k:k + 1], sub.det_rows, sub.det_cols, sub.R, sub.T)
            mu, _ = ref.Oracle(one).sart(data64[k:k + 1], mu, 1, lam, vox_weights=wts, nthreads=nthreads)
        ref_iters.append(mu.copy())
    log("mixed: oracle iterates (12 views x 2) in %.1f s" % (time.perf_counter() - t0))
    Gs = cyl.Geometry(sub, 0)
    for name, tdt in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        p = data.to(tdt).contiguous()
        vol = torch.from_numpy(ph.prior.astype(np.float32)).cuda().to(tdt).contiguous()
        w = torch.from_numpy(wts).cuda().to(tdt).contiguous()
        errs = []
        for it in range(2):
            Gs.sart(p, vol, it + 1, lam, vox_weights=w, start_iter=it)
            got = vol.float().cpu().numpy().astype(np.float64).ravel()
            want = np.ravel(ref_iters[it])
            errs.append(float(np.linalg.norm(got - want) / np.linalg.norm(want)))
        out.setdefault(name, {})
        out[name]["rel_l2_vs_fp64_oracle"] = errs
        out[name]["final_rel_l2_vs_fp64_oracle"] = errs[-1]
        log("mixed %s: rel L2 vs FP64 oracle per iteration %s" % (name, " ".join("%.3e" % e for e in errs)))
    out["accuracy_run"] = "256x720x128 grid, 12 of the 120 views (every 10th), 2 weighted SART iterations from the prior"
    out["storage"] = "volume, projections and voxel weights in the named type; FP32 arithmetic and residual images"
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2005_11976_amd import cyl, inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cyl.lib()
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    cfg = I.config_single()
    scan = cfg["scan"]
    g = scan.grid
    log("config", cfg["name"], g.shape, scan.proj_shape, "dtype", args.dtype)
    ph = I.industrial_phantom(g, cfg["seed"])
    G = cyl.Geometry(scan, 0)
    truth = torch.from_numpy(ph.truth.astype(np.float32)).cuda()
    # measured line integrals: forward projection of the truth (synthetic data)
    p32 = G.fp(truth)
    p = p32.to(tdt).contiguous()
    prior = torch.from_numpy(ph.prior.astype(np.float32)).cuda().to(tdt).contiguous()
    w = torch.from_numpy(ph.weights.astype(np.float32)).cuda().to(tdt).contiguous()
    ws = torch.empty(G.workspace_bytes(), dtype=torch.uint8, device="cuda")
    vol = prior.clone()
    torch.cuda.synchronize()

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        G.sart(p, vol, 1, cfg["lam"], vox_weights=w, workspace=ws)
    torch.cuda.synchronize()
    vol.copy_(prior)
    torch.cuda.synchronize()

    log("timed", args.steps, "steps")
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for s in range(args.steps):
        G.sart(p, vol, s + 1, cfg["lam"], vox_weights=w, workspace=ws, start_iter=s)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    it_s = 1000.0 / ms_per_step
    rays = scan.n_views * scan.det_rows * scan.det_cols
    grays = 2.0 * rays * it_s / 1e9
    log("SART %.3f it/s  %.2f ms/iter  %.3f Grays/s (wall %.2f s)" % (it_s, ms_per_step, grays, wall))

    # reconstruction quality vs the truth (reported, not a parity claim)
    rel_truth = float((vol.float() - truth).norm() / truth.norm())

    # per-kernel HIP-event timing on the launch stream
    nk = min(args.kernel_views, scan.n_views)
    log("kernel timing over", nk, "views")
    vol2 = prior.clone()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(3 * nk)]
    for i in range(nk):
        evs[3 * i].record()
        G.sart_residual(i, p, vol2, ws)
        evs[3 * i + 1].record()
        G.sart_update(i, vol2, ws, cfg["lam"], vox_weights=w)
        evs[3 * i + 2].record()
    torch.cuda.synchronize()
    fp_ms = float(np.mean([evs[3 * i].elapsed_time(evs[3 * i + 1]) for i in range(nk)]))
    bp_ms = float(np.mean([evs[3 * i + 1].elapsed_time(evs[3 * i + 2]) for i in range(nk)]))
    log("kernel avg ms: fp_residual %.4f  bp_update %.4f" % (fp_ms, bp_ms))

    s_mu = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    V = g.n_vox
    P = scan.det_rows * scan.det_cols
    # algorithmic bytes per launch (one view): FP reads mu and p, writes rho;
    # BP reads rho, reads mu and w, writes mu
    fp_bytes = V * s_mu + P * (s_mu + 4)
    bp_bytes = P * 4 + V * (2 * s_mu + s_mu)
    dom = "bp_update" if bp_ms >= fp_ms else "fp_residual"
    dom_bytes = bp_bytes if dom == "bp_update" else fp_bytes
    dom_ms = max(bp_ms, fp_ms)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    if args.dtype == "f32" and kernel_src_sha() == MEASURED_TRAFFIC["src_sha"]:
        traffic = MEASURED_TRAFFIC[dom]
    valu = None
    if args.dtype == "f32" and kernel_src_sha() == MEASURED_VALU["src_sha"]:
        valu = {k: {"instructions_per_launch": MEASURED_VALU[k],
                    "issue_frac": MEASURED_VALU[k] / (VALU_ISSUE_PER_S * ms * 1e-3),
                    "active_lanes": MEASURED_VALU["active_lanes"][k]}
                for k, ms in (("fp_residual", fp_ms), ("bp_update", bp_ms))}
    iter_bytes = scan.n_views * (fp_bytes + bp_bytes)
    path_gbs = iter_bytes * it_s / 1e9

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    os_out = None if args.core_only else ordered_subsets(G, scan, p, prior, w, cfg["lam"], truth)
    cmp_out = None if args.core_only or args.dtype != "f32" else comparison_projectors(
        G, scan, p, prior, w, cfg["lam"], truth)
    sym_out = None if args.core_only else symmetric_matrix(G, scan, p, prior, w, cfg["lam"], truth)
    pose_out = None if args.core_only else pose_estimation(scan)
    rates_out = None if args.core_only or args.dtype != "f32" else projector_rates(G, scan, truth, p32)
    large_out = None if args.core_only or args.dtype != "f32" else posed_large()
    serving_out = serving(args) if args.serve_requests > 0 and not args.core_only else None

    nthreads = max(1, min(16, len(os.sched_getaffinity(0))))
    mixed_out = None
    if not args.core_only and not args.no_mixed and args.dtype == "f32":
        mixed_out = mixed_precision(cfg, ph, p32, nthreads)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on", nthreads, "threads")
        cpu = cpu_baseline(scan, ph.truth, ph.prior, ph.weights, p32.cpu().numpy(), nthreads)
        log("cpu baseline %.5f it/s" % cpu["value"])

    out = {
        "metric": "SART iters/s (weighted, from prior) at 256x720x128, 120 views of 512x512",
        "value": it_s,
        "unit": "SART it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": list(g.shape), "views": scan.n_views,
                   "detector": [scan.det_rows, scan.det_cols], "iterations_per_step": 1,
                   "lambda": cfg["lam"], "weighted": True, "prior": True},
        "grays_per_s_fwd_bp": grays,
        "path_hbm_gbs_algorithmic": path_gbs,
        "path_hbm_frac": path_gbs / HBM_PEAK_GBS,
        "kernel_ms": {"fp_residual": fp_ms, "bp_update": bp_ms},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": dom_bytes},
        "valu": valu,
        "cpu_baseline": cpu,
        "mixed": mixed_out,
        "ordered_subsets": os_out,
        "comparison_projectors": cmp_out,
        "symmetric_matrix": sym_out,
        "serving": serving_out,
        "projector_rates": rates_out,
        "posed_large": large_out,
        "pose_estimation": pose_out,
        "rel_err_vs_truth": rel_truth,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
