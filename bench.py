#!/usr/bin/env python3
"""Benchmark: seed-scale window evaluations per second on the PET-like workload.

One step = one full detection pass over the resident 128x128x64 uint16 PET-like
volume (64 bins, seed spacing 6, scales 4..16, 50 iterations) with both methods:
quadrant ascent and mean-shift toward the uniform pmf (range scan, binning,
persistent searches with the final saliency pass, device ranking, results to
host).  The input is in HBM before the timed region starts.

Prints one JSON line.  Extra fields: volumes/s, per-method device times, the
roofline of the dominant kernel (the mean-shift search) measured with HIP events
on the launch stream (against the published HBM peak and the measured copy
peak), both searches' LDS-atomic rates against measured LDS ceilings, the
host-to-device copy of the volume (outside the timed step), the every-voxel
saliency map against the seed-grid detection, the CPU oracle timed
on a bounded sample, the uneven 64-volume batch (one captured launch sequence)
against plain per-volume launches, and Poisson serving streams at several rates
against a plain one-launch-per-volume loop with p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X fp64 vector, published


SECTIONS = ("dense_map", "window_level", "tracking", "abmsod")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-stride", type=int, default=1)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_k_search_ms_pet128x128x64.json"))
    ap.add_argument("--abmsod-ops-json", default=os.path.join(ROOT, "profiles", "alu_k_abmsod_pet128x128x64.json"))
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed step and the roofline microbenchmarks (for profiling runs)")
    ap.add_argument("--section", choices=SECTIONS,
                    help="run only this one extra section and print its record (for profiling runs)")
    return ap.parse_args()


def batch_section(ks, torch, ctx):
    """The 64-volume uneven batch: one ks_detect_batch (captured graph, replayed)
    against one ks_detect_device per volume, same volumes, same results."""
    from paper_1310_6736_amd import synth

    ws = synth.batch_workloads()
    vols = [torch.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    cap = 256
    ks.ks_detect_batch(ctx, reqs, capacity=cap)  # capture
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        res_b = ks.ks_detect_batch(ctx, reqs, capacity=cap)
    tb = (time.perf_counter() - t0) / reps
    for v, w in zip(vols, ws):  # warm
        ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res_p = [ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
                 for v, w in zip(vols, ws)]
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
    same = all(a[1] == b[1] and np.array_equal(a[0], b[0]) for a, b in zip(res_b, res_p))
    return {"workload": "64 volumes, x,y in 64..192, z in 64..128, types 50/30/20 (spheres u8 / PET-like u16 / "
                        "MR-like i16), per-type bins, spacing, scales and method",
            "batched_volumes_per_s": len(ws) / tb, "plain_volumes_per_s": len(ws) / tp,
            "batched_ms": tb * 1e3, "plain_ms": tp * 1e3, "speedup": tp / tb, "identical_results": bool(same)}


def serving_section(ks, torch, ctx, n_req):
    """Poisson streams of the 50/30/20 mix at native sizes: the continuous-batching
    server against a plain loop that serves requests one launch sequence at a
    time in arrival order (both copy each host volume to the device).  Arrival
    rates 0.5, 0.7, 0.9 and 1.2 x the plain loop's measured capacity, a saturated
    stream (all requests at t = 0), and the saturated stream under a budget that
    holds one large request at a time."""
    from paper_1310_6736_amd import synth

    pool = {0: [synth.typed_workload(0, 2000 + i, synth.TYPE_DIMS[0]) for i in range(4)],
            1: [synth.typed_workload(1, 2100 + i, synth.TYPE_DIMS[1], method_parity=i) for i in range(4)],
            2: [synth.typed_workload(2, 2200 + i, synth.TYPE_DIMS[2]) for i in range(2)]}
    cap = 64
    tdt = {np.dtype(np.uint8): torch.uint8, np.dtype(np.int16): torch.int16,
           np.dtype(np.uint16): getattr(torch, "uint16", None)}
    dev_buf = {k: [torch.empty(w.volume.shape, dtype=tdt[w.volume.dtype], device="cuda:0") for w in ws]
               for k, ws in pool.items()}

    def plain_one(kind, j):
        w = pool[kind][j]
        d = dev_buf[kind][j]
        d.copy_(torch.from_numpy(w.volume))
        return ks.ks_detect_device(ctx, d, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)

    # plain capacity on the mix (saturated, arrival order)
    trace = synth.arrival_trace(1.0, n=n_req)
    order = [(k, (seed % len(pool[k]))) for _, k, seed, _ in trace]
    for k, j in order[:8]:
        plain_one(k, j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, j in order:
        plain_one(k, j)
    torch.cuda.synchronize()
    c_plain = n_req / (time.perf_counter() - t0)

    def run_plain(trace):
        lat = []
        start = time.perf_counter()
        for t_arr, k, seed, _ in trace:
            now = time.perf_counter() - start
            if now < t_arr:
                time.sleep(t_arr - now)
            plain_one(k, seed % len(pool[k]))
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - start - t_arr) * 1e3)
        span = time.perf_counter() - start
        return {"volumes_per_s": len(trace) / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(np.mean(lat))}

    def run_server(srv, trace):
        srv.reset_stats()
        tickets = []
        start = time.perf_counter()
        for t_arr, k, seed, _ in trace:
            now = time.perf_counter() - start
            if now < t_arr:
                time.sleep(t_arr - now)
            w = pool[k][seed % len(pool[k])]
            tickets.append(srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter))
        srv.drain()
        st = srv.stats()
        for t in tickets:
            srv.poll(t, capacity=cap)
        return {"volumes_per_s": st["volumes_per_s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "mean_ms": st["mean_ms"], "refused": int(st["refused"])}

    sat = [(0.0, k, seed, i) for _, k, seed, i in trace]
    out = {"workload": "%d requests, Poisson arrivals, 50/30/20 mix of the 64^3 spheres, 128x128x64 PET-like "
                       "(quadrant/mean-shift alternating) and 256x256x160 MR-like generators" % n_req,
           "plain_capacity_volumes_per_s": c_plain}
    srv = ks.Server(0, hbm_budget=8 << 30, max_slots=4)
    run_server(srv, sat)  # warm-up: the slots' device buffers grow to the mix's sizes
    out["saturated"] = {"server": run_server(srv, sat), "plain": run_plain(sat)}
    for f in (0.5, 0.7, 0.9, 1.2):
        lam = f * c_plain
        tr = synth.arrival_trace(lam, n=n_req)
        out["rate_%.1f" % f] = {"rate_per_s": lam, "server": run_server(srv, tr), "plain": run_plain(tr)}
    srv.close()
    # a budget that holds one MR-like request (about 130 MB of device state) at a time
    small = 160 << 20
    srv = ks.Server(0, hbm_budget=small, max_slots=4)
    run_server(srv, sat[:16])
    out["small_budget"] = {"budget_bytes": small, "saturated": run_server(srv, sat)}
    srv.close()
    return out


def dense_section(ks, torch, ctx, q_detect_ms):
    """The every-voxel Kadir-Brady map (the search the seed grid replaces) on the
    spheres and PET-like volumes, against the seed-grid quadrant detection of the
    same volume and scales: the seed grid's saving measured on this GPU."""
    from paper_1310_6736_amd import synth

    ks.ks_context_set_profiling(ctx, True)
    out = {}
    for w, det in ((synth.spheres_64(), None), (synth.pet_shell(ks.KS_QUADRANT), q_detect_ms)):
        v = torch.from_numpy(w.volume).to("cuda:0")
        ks.ks_saliency_map(ctx, v, w.bins, w.scales)
        ts = []
        for _ in range(3):
            ks.ks_saliency_map(ctx, v, w.bins, w.scales)
            ts.append(ks.ks_last_stats(ctx)["ms_search"])
        if det is None:
            dts = []
            for _ in range(5):
                ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=64)
                dts.append(ks.ks_last_stats(ctx)["ms_total"])
            det = float(np.median(dts))
        m = float(np.median(ts))
        out[w.name] = {"voxels": int(w.volume.size), "scales": list(w.scales), "map_ms": m,
                       "seed_grid_detect_ms": det, "saving": m / det}
    ks.ks_context_set_profiling(ctx, False)
    return out


def window_level_section(ks, torch, ctx):
    """Constrained-range entropy (window level) on the MR-like volume: the
    mean-shift detection binned over the lesion window only, against the same
    detection over the full dynamic range."""
    from paper_1310_6736_amd import synth

    w = synth.mr_blobs()
    v = torch.from_numpy(w.volume).to("cuda:0")
    out = {"workload": w.name, "window": [1201, 3000]}
    ks.ks_context_set_profiling(ctx, True)
    try:
        for name, opt in (("full_range", None), ("window", ks.options(window=(1201, 3000)))):
            ks.ks_context_set_options(ctx, opt)
            ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=64)
            ts, n, st = [], 0, None
            for _ in range(3):
                _, n = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=64)
                st = ks.ks_last_stats(ctx)
                ts.append(st["ms_total"])
            m = float(np.median(ts))
            out[name] = {"device_ms": m, "regions": int(n), "window_evals": int(st["window_evals"]),
                         "window_evals_per_s": st["window_evals"] / (m * 1e-3)}
    finally:
        ks.ks_context_set_options(ctx, None)
        ks.ks_context_set_profiling(ctx, False)
    return out


def tracking_section(ks, torch, ctx, n_frames=5, max_seeds=20):
    """Warm start from the previous frame's regions: PET-like frames in which the
    volume moves one voxel along x per frame.  Every frame runs the seed grid, and
    every frame after the first also runs a warm start from the first max_seeds
    distinct positions of the previous frame's warm (frame 0: grid) regions."""
    from paper_1310_6736_amd import synth

    w = synth.pet_shell(ks.KS_QUADRANT)
    frames = [torch.from_numpy(np.ascontiguousarray(np.roll(w.volume, f, axis=2))).to("cuda:0")
              for f in range(n_frames)]

    def run(v, seeds):
        ks.ks_context_set_seeds(ctx, seeds)
        regs, n = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
        return regs, n, ks.ks_last_stats(ctx)

    def top(regs, n):
        return [int(regs[f][0]) for f in ("x", "y", "z", "scale")] + [float(regs["saliency"][0])] if n else None

    ks.ks_context_set_profiling(ctx, True)
    grid_ms, warm_ms, warm_traj, grid_top, warm_top = [], [], [], [], []
    try:
        for rep in range(2):
            prev = None
            for f, v in enumerate(frames):
                g, gn, gst = run(v, None)
                regs, n = g, gn
                if f > 0:
                    pts = []
                    for r in prev:
                        p = (int(r["x"]), int(r["y"]), int(r["z"]))
                        if p not in pts:
                            pts.append(p)
                        if len(pts) == max_seeds:
                            break
                    regs, n, st = run(v, np.array(pts, np.int32) if pts else None)
                    if rep == 1:
                        warm_ms.append(st["ms_total"])
                        warm_traj.append(int(st["trajectories"]))
                        warm_top.append(top(regs, n))
                if rep == 1:
                    grid_ms.append(gst["ms_total"])
                    grid_top.append(top(g, gn))
                prev = regs
    finally:
        ks.ks_context_set_seeds(ctx, None)
        ks.ks_context_set_profiling(ctx, False)
    gm, wm = float(np.median(grid_ms)), float(np.median(warm_ms))
    return {"workload": w.name + " moved 1 voxel/frame along x", "frames": n_frames, "max_seeds": max_seeds,
            "grid_frame_ms": gm, "warm_frame_ms": wm, "speedup": gm / wm, "warm_trajectories": warm_traj,
            "grid_top_region": grid_top, "warm_top_region": warm_top[:],
            "warm_top_saliency_over_grid_top": [a[4] / b[4] if a and b else None
                                                for a, b in zip(warm_top, grid_top[1:])]}


def abmsod_section(ks, torch, ctx, ops_json):
    """ABMSOD (ellipsoidal Gaussian-weighted windows with bandwidth updates) on the
    PET-like volume: every grid seed x every start radius 4..16, 20 iterations.
    Bound by fp64 arithmetic: the fp64 operations per window voxel come from the
    committed counter summary (None once the kernel sources have changed)."""
    from paper_1310_6736_amd import synth

    w = synth.pet_shell(ks.KS_QUADRANT)
    radii, max_iter = (4, 16), 20
    v = torch.from_numpy(w.volume).to("cuda:0")
    ks.ks_context_set_profiling(ctx, True)
    try:
        out = ks.ks_abmsod(ctx, v, w.bins, w.spacing, radii, max_iter)
        ts, st = [], None
        for _ in range(3):
            out = ks.ks_abmsod(ctx, v, w.bins, w.spacing, radii, max_iter)
            st = ks.ks_last_stats(ctx)
            ts.append(st["ms_search"])
    finally:
        ks.ks_context_set_profiling(ctx, False)
    m = float(np.median(ts))
    visits_per_s = st["voxel_visits"] / (m * 1e-3)
    ops = measured_record(ops_json, "fp64_ops_per_visit")
    line = {"workload": w.name + ", radii 4..16, 20 iterations, threshold 0", "kernel": "k_abmsod",
            "candidates": int(len(out)), "device_ms": m, "window_histograms": int(st["evals"]),
            "window_voxel_visits": int(st["voxel_visits"]), "visits_per_s": visits_per_s,
            "mean_iterations": float(out["iters"].mean()),
            "stops": {k: int(n) for k, n in zip(("max_iter", "converged", "deteriorated", "empty", "degenerate"),
                                                np.bincount(out["stop"], minlength=5))}}
    achieved = None if ops is None else ops * visits_per_s / 1e12
    line["roofline"] = {"bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS, "achieved": achieved,
                        "frac": None if achieved is None else achieved / FP64_PEAK_TFLOPS,
                        "fp64_ops_per_visit": ops}
    return line


def measured_record(path, field):
    """A field of a committed counter summary, or None when the kernel sources
    have changed since the counters were taken (the summary records a SHA-256 of
    the files that define the kernel)."""
    import hashlib

    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["source_files"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return rec[field]
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(path):
    """HBM bytes per launch of the mean-shift search from the committed counter
    summary, or None when the kernel sources have changed since then."""
    return measured_record(path, "bytes_per_launch")


def _oracle_shard(job):
    """One worker of the CPU baseline: the oracle on one interleaved share of the
    trajectory ids of one method."""
    import oracle
    from paper_1310_6736_amd import synth

    method, stride, worker, workers = job
    w = synth.pet_shell(method)
    n = oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)
    ids = np.arange(0, n, stride, dtype=np.int64)[worker::workers]
    _, st = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
    return st["window_evals"], len(ids), n


def cpu_baseline(stride: int, workers: int):
    """The oracle as it stands on every stride-th trajectory of the same workload,
    sharded over `workers` processes by trajectory id; window evaluations per
    second of wall time.  Runs before the GPU is initialised (the pool forks)."""
    import multiprocessing as mp

    jobs = [(m, stride, k, workers) for m in (0, 1) for k in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_shard, jobs, chunksize=1)
    total_s = time.perf_counter() - t0
    total_evals = sum(r[0] for r in res)
    done = {m: sum(r[1] for r, j in zip(res, jobs) if j[0] == m) for m in (0, 1)}
    of = {m: next(r[2] for r, j in zip(res, jobs) if j[0] == m) for m in (0, 1)}
    which = "every trajectory" if stride == 1 else "every %d-th trajectory" % stride
    return {"value": total_evals / total_s, "unit": "window_evals/s", "cores": workers, "kind": "oracle",
            "sample": "%s of the PET-like volume, both methods (quadrant %d/%d, mean-shift %d/%d trajectories), "
                      "ids dealt round-robin to %d processes; %.1f s wall" %
                      (which, done[0], of[0], done[1], of[1], workers, total_s)}


def section_only(name):
    """One extra section alone, on a fresh context: the workload of a kernel-trace
    profile of that section."""
    import torch

    from paper_1310_6736_amd import ks

    ctx = ks.Context(0)
    if name == "dense_map":
        rec = dense_section(ks, torch, ctx, None)
    elif name == "window_level":
        rec = window_level_section(ks, torch, ctx)
    elif name == "tracking":
        rec = tracking_section(ks, torch, ctx)
    else:
        rec = abmsod_section(ks, torch, ctx, os.path.join(ROOT, "profiles", "alu_k_abmsod_pet128x128x64.json"))
    ctx.close()
    print(json.dumps({"section": name, name: rec}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.section:
        section_only(args.section)
        return
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample_stride, max(1, min(16, os.cpu_count() or 1)))
    import torch

    from paper_1310_6736_amd import ks, synth

    dev = torch.device("cuda:0")
    ctx = ks.Context(0)
    wq = synth.pet_shell(ks.KS_QUADRANT)
    wm = synth.pet_shell(ks.KS_MEANSHIFT)
    vol = torch.from_numpy(wq.volume).to(dev)
    stream = torch.cuda.current_stream()
    cap = 1024

    # Each method alone first: the per-search work counters (deterministic, the
    # same in the batched step) and the searches' isolated launch times.
    ks.ks_context_set_profiling(ctx, True)
    iso = {}
    for w in (wq, wm):
        ts = []
        for _ in range(max(3, args.warmup)):
            _, n = ks.ks_detect_device(ctx, vol, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap,
                                       stream=stream)
            st = ks.ks_last_stats(ctx)
            ts.append(st["ms_search"])
        iso[w.method] = {"regions": n, "stats": st, "search_ms": float(np.median(ts)), "total_ms": st["ms_total"]}
    ks.ks_context_set_profiling(ctx, False)

    # The step: both methods on the volume in one batched call; the two searches
    # run concurrently on two streams.
    reqs = [ks.make_request(vol, w.bins, w.spacing, w.scales, w.method, w.max_iter) for w in (wq, wm)]

    def step(profile_sink=None):
        res = ks.ks_detect_batch(ctx, reqs, capacity=cap, stream=stream)
        if profile_sink is not None:
            profile_sink.append(ks.ks_last_stats(ctx))
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ks.ks_context_set_profiling(ctx, True)
    prof = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step(prof)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks.ks_context_set_profiling(ctx, False)

    window_evals = prof[-1]["window_evals"]
    ms_per_step = dt * 1000.0 / args.steps
    ms_iso, q_iso = iso[ks.KS_MEANSHIFT]["stats"], iso[ks.KS_QUADRANT]["stats"]
    assert window_evals == ms_iso["window_evals"] + q_iso["window_evals"]
    ms_kernel_ms = float(np.mean([s["ms_search_ms"] for s in prof]))
    q_kernel_ms = float(np.mean([s["ms_search_quad"] for s in prof]))
    ms_bytes = ms_iso["voxel_visits"] + ms_iso["final_visits"]
    q_bytes = q_iso["voxel_visits"] + q_iso["final_visits"]
    achieved = ms_bytes / (ms_kernel_ms * 1e-3) / 1e9
    achieved_iso = ms_bytes / (iso[ks.KS_MEANSHIFT]["search_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json)
    # measured ceilings: streaming copy, conflict-free 64-bit / 32-bit LDS atomics
    copy_gbs = ks.ks_roofline(ks.KS_ROOF_COPY) / 1e9
    lds64 = ks.ks_roofline(ks.KS_ROOF_LDS_ADD64)
    lds32 = ks.ks_roofline(ks.KS_ROOF_LDS_ADD32)
    ms_ops, q_ops = float(ms_iso["lds_ops"]), float(q_iso["lds_ops"])
    ms_swept = float(ms_iso["swept_voxels"])
    ms_iso_ms, q_iso_ms = iso[ks.KS_MEANSHIFT]["search_ms"], iso[ks.KS_QUADRANT]["search_ms"]
    # host-to-device copy of the input volume (not part of the timed step)
    host = torch.from_numpy(wq.volume)
    pinned = host.pin_memory()
    h2d = {}
    for name, src in (("pageable", host), ("pinned", pinned)):
        buf = torch.empty_like(vol)
        buf.copy_(src)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(10):
            buf.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        h2d[name + "_ms"] = (time.perf_counter() - t1) * 100.0

    line = {
        "metric": "seed-scale window evals/sec",
        "value": window_evals / (dt / args.steps),
        "unit": "window_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8 bins, int32 counts, f64 decisions, f32 saliency",
        "data": "synthetic",
        "config": {"workload": "PET-like 128x128x64 uint16 ellipsoidal shell, 64 bins, seed spacing 6, "
                               "scales 4..16, max 50 iterations, quadrant + mean-shift in one batched call "
                               "(the two searches concurrent)",
                   "trajectories": {"quadrant": int(q_iso["trajectories"]),
                                    "meanshift": int(ms_iso["trajectories"])}},
        "volumes_per_s": 1000.0 / ms_per_step,
        "regions": {"quadrant": int(res[0][1]), "meanshift": int(res[1][1])},
        "window_evals_per_step": int(window_evals),
        "device_ms": {"search_phase": float(np.mean([s["ms_search"] for s in prof])),
                      "quadrant_search": q_kernel_ms, "meanshift_search": ms_kernel_ms,
                      "prep_ms": float(np.mean([s["ms_prep"] for s in prof])),
                      "rank_ms": float(np.mean([s["ms_rank"] for s in prof])),
                      "isolated": {"quadrant_search": q_iso_ms, "meanshift_search": ms_iso_ms}},
        # the mean-shift search's launches in the timed step, which share the GPU with
        # the quadrant search for most of their duration; "isolated": the same launch
        # alone on the GPU (before the timed region)
        "roofline": {"bound": "hbm", "kernel": "k_search_ms", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": int(ms_bytes),
                     "swept_bytes_per_launch": int(ms_swept),
                     "copy_peak_measured": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "concurrent_with": "k_search_quad",
                     "isolated": {"device_ms": ms_iso_ms, "achieved": achieved_iso,
                                  "frac": achieved_iso / HBM_PEAK_GBS,
                                  "frac_of_measured_copy": achieved_iso / copy_gbs},
                     "search_phase_achieved": (ms_bytes + q_bytes) / (np.mean([s["ms_search"] for s in prof]) * 1e-3) / 1e9,
                     "quadrant_achieved": q_bytes / (q_kernel_ms * 1e-3) / 1e9,
                     "quadrant_isolated_achieved": q_bytes / (q_iso_ms * 1e-3) / 1e9},
        "lds_atomic": {"unit": "lane-ops/s",
                       "meanshift": {"kernel": "k_search_ms", "ops_per_launch": int(ms_ops),
                                     "achieved": ms_ops / (ms_kernel_ms * 1e-3), "peak": lds64,
                                     "peak_kind": "conflict-free 64-bit LDS add microbenchmark",
                                     "frac": ms_ops / (ms_kernel_ms * 1e-3) / lds64,
                                     "isolated_frac": ms_ops / (ms_iso_ms * 1e-3) / lds64},
                       "quadrant": {"kernel": "k_search_quad", "ops_per_launch": int(q_ops),
                                    "achieved": q_ops / (q_kernel_ms * 1e-3), "peak": lds32,
                                    "peak_kind": "conflict-free 32-bit LDS add microbenchmark",
                                    "frac": q_ops / (q_kernel_ms * 1e-3) / lds32,
                                    "isolated_frac": q_ops / (q_iso_ms * 1e-3) / lds32}},
        "h2d": dict(h2d, bytes=int(wq.volume.nbytes),
                    pcie_inclusive_window_evals_per_s=window_evals / (dt / args.steps + h2d["pinned_ms"] * 1e-3)),
    }
    q_total = iso[ks.KS_QUADRANT]["total_ms"]
    if not args.main_only:
        line["dense_map"] = dense_section(ks, torch, ctx, q_total)
        line["window_level"] = window_level_section(ks, torch, ctx)
        line["tracking"] = tracking_section(ks, torch, ctx)
        line["abmsod"] = abmsod_section(ks, torch, ctx, args.abmsod_ops_json)
    if not (args.no_batch or args.main_only):
        line["batch"] = batch_section(ks, torch, ctx)
    if not (args.no_serve or args.main_only):
        line["serving"] = serving_section(ks, torch, ctx, args.serve_requests)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
