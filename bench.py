#!/usr/bin/env python3
"""Benchmark: seed-scale window evaluations per second on the MR-like workload.

One step = one full mean-shift detection (Sec. 2.3) of the resident 256x256x160
int16 MR-like volume (64 bins, seed spacing 8, scales 4..24: 430,080
trajectories, 100 iterations): range scan, binning, the persistent search with
the final saliency pass, device ranking of every trajectory, the top regions to
host, as one replay of the library's captured graph.  The input is in HBM
before the timed region starts.

Prints one JSON line.  Extra fields: volumes/s, device times per phase, the
roofline of the dominant kernel (the mean-shift search, timed by event-record
nodes around it inside each replayed graph) as algorithmic, swept and
LDS-atomic fractions with the counters that show what binds it, the CPU oracle
on a bounded sample of the same workload (all host cores and one pinned core),
the PET-like 128x128x64 workload (both methods in one batched call), the
every-voxel saliency map against the seed-grid detection, the window level, the
tracking warm start, ABMSOD, the uneven 64-volume batch against plain
per-volume launches, and Poisson serving streams against a plain
one-launch-per-volume loop with p50/p99 latency.
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


SECTIONS = ("dense_map", "window_level", "tracking", "abmsod", "pet_like", "batch", "serving")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-stride", type=int, default=16,
                    help="CPU baseline on every n-th grid seed (all scales), all host cores")
    ap.add_argument("--cpu-single-stride", type=int, default=64,
                    help="CPU baseline on every n-th grid seed (all scales), one pinned core")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_k_search_ms_mr256x256x160.json"))
    ap.add_argument("--counters-json", default=os.path.join(ROOT, "profiles", "counters_k_search_ms_mr256x256x160.json"))
    ap.add_argument("--abmsod-ops-json", default=os.path.join(ROOT, "profiles", "alu_k_abmsod_pet128x128x64.json"))
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed MR-like step and the roofline microbenchmarks (for profiling runs)")
    ap.add_argument("--section", choices=SECTIONS,
                    help="run only this one extra section and print its record (for profiling runs)")
    return ap.parse_args()


def batch_section(ks, torch, ctx):
    """The 64-volume uneven batch: one ks_detect_batch (captured graph, replayed)
    against one ks_detect_device per volume, same volumes, same results; the
    batch with the context's default shapes and with the shapes
    ks_context_autotune_batch picks for it (on a context of its own)."""
    from paper_1310_6736_amd import synth

    ws = synth.batch_workloads()
    vols = [torch.from_numpy(w.volume).to("cuda:0") for w in ws]
    torch.cuda.synchronize()
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    cap = 256
    reps = 3

    def timed_batch(c):
        ks.ks_detect_batch(c, reqs, capacity=cap)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = ks.ks_detect_batch(c, reqs, capacity=cap)
        return (time.perf_counter() - t0) / reps, res

    tb, res_b = timed_batch(ctx)
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
    tctx = ks.Context(0)
    t0 = time.perf_counter()
    tuning = ks.ks_context_autotune_batch(tctx, reqs, reps=2)
    tune_s = time.perf_counter() - t0
    ta, res_a = timed_batch(tctx)
    same_a = all(a[1] == b[1] and np.array_equal(a[0], b[0]) for a, b in zip(res_a, res_p))
    tctx.close()
    return {"workload": "64 volumes, x,y in 64..192, z in 64..128, types 50/30/20 (spheres u8 / PET-like u16 / "
                        "MR-like i16), per-type bins, spacing, scales and method",
            "batched_volumes_per_s": len(ws) / ta, "plain_volumes_per_s": len(ws) / tp,
            "batched_ms": ta * 1e3, "plain_ms": tp * 1e3, "speedup": tp / ta,
            "identical_results": bool(same and same_a),
            "autotuned": {"tuning": dict(zip(("ms_replicas_log2", "ms_small_replicas_log2", "s_small",
                                               "quad_replicas_log2", "ms_scales_per_task"), tuning)),
                          "tuning_seconds": tune_s, "batched_ms": ta * 1e3},
            "default_shapes": {"batched_volumes_per_s": len(ws) / tb, "batched_ms": tb * 1e3}}


def _stream_volume(job):
    """Volume of request i of the serving stream: generator type `kind` at its
    native size, volume seed 2000 + i (type-1 requests alternate methods)."""
    from paper_1310_6736_amd import synth

    kind, seed, parity = job
    return synth.typed_workload(kind, seed, synth.TYPE_DIMS[kind], method_parity=parity)


def stream_workloads(n_req, workers):
    """One volume per request of the serving stream (the type sequence is the
    same at every arrival rate), generated on the host cores before the GPU is
    initialised (the pool forks)."""
    import multiprocessing as mp

    from paper_1310_6736_amd import synth

    jobs = [(k, seed, parity) for _, k, seed, parity in synth.arrival_trace(1.0, n=n_req)]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_stream_volume, jobs, chunksize=1)


def serving_section(ks, torch, ctx, ws):
    """Poisson streams of the 50/30/20 mix at native sizes, one volume per
    request: the continuous-batching server against a plain loop that serves
    requests one launch sequence at a time in arrival order (both copy each host
    volume to the device).  Arrival rates 0.5, 0.7, 0.9 and 1.2 x the plain
    loop's measured capacity, a saturated stream (all requests at t = 0), and the
    saturated stream under a budget that holds one large request at a time."""
    from paper_1310_6736_amd import synth

    n_req = len(ws)
    cap = 64
    tdt = {np.dtype(np.uint8): torch.uint8, np.dtype(np.int16): torch.int16,
           np.dtype(np.uint16): getattr(torch, "uint16", None)}
    dev_buf = {}
    for w in ws:
        key = (w.volume.shape, w.volume.dtype)
        if key not in dev_buf:
            dev_buf[key] = torch.empty(w.volume.shape, dtype=tdt[w.volume.dtype], device="cuda:0")

    def plain_one(i):
        w = ws[i]
        d = dev_buf[(w.volume.shape, w.volume.dtype)]
        d.copy_(torch.from_numpy(w.volume))
        return ks.ks_detect_device(ctx, d, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)

    # plain capacity on the mix (saturated, arrival order)
    for i in range(8):
        plain_one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_req):
        plain_one(i)
    torch.cuda.synchronize()
    c_plain = n_req / (time.perf_counter() - t0)

    def run_plain(trace):
        lat = []
        start = time.perf_counter()
        for t_arr, _, _, i in trace:
            now = time.perf_counter() - start
            if now < t_arr:
                time.sleep(t_arr - now)
            plain_one(i)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - start - t_arr) * 1e3)
        span = time.perf_counter() - start
        return {"volumes_per_s": len(trace) / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(np.mean(lat))}

    def run_server(srv, trace):
        srv.reset_stats()
        tickets = []
        start = time.perf_counter()
        for t_arr, _, _, i in trace:
            now = time.perf_counter() - start
            if now < t_arr:
                time.sleep(t_arr - now)
            w = ws[i]
            tickets.append(srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, max_regions=cap))
        srv.drain()
        st = srv.stats()
        for t in tickets:
            srv.poll(t, capacity=cap)
        return {"volumes_per_s": st["volumes_per_s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "mean_ms": st["mean_ms"], "refused": int(st["refused"]), "peak_device_bytes": int(st["bytes_peak"])}

    sat = [(0.0, k, seed, i) for _, k, seed, i in synth.arrival_trace(1.0, n=n_req)]
    out = {"workload": "%d requests, Poisson arrivals, 50/30/20 mix of the 64^3 spheres, 128x128x64 PET-like "
                       "(quadrant/mean-shift alternating) and 256x256x160 MR-like generators, one volume per "
                       "request (volume seed 2000 + i)" % n_req,
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


# Algorithmic fp64 operations of one ABMSOD iteration per counted window voxel
# (Sec. 2.3 Alg. 2).  Every sweep tests membership, u = v - x and
# u^T H^-1 u: 3 + 18 operations.  The histogram-and-mean sweep then takes
# g = exp(-d/2) (2), its fixed-point scaling (1) and the three weighted offsets
# (6): 30 for a voxel it counts twice (histogram and mean), 15 per visit.  The
# histogram sweep at x_new: 21 + 3 = 24.  The covariance sweep (Eq. 7): the bin
# weight and six products-and-sums, 21 + 19 = 40.  Four visits per iteration:
# (30 + 24 + 40) / 4.
ABM_ALG_OPS_PER_VISIT = (30 + 24 + 40) / 4.0


def abmsod_section(ks, torch, ctx, ops_json):
    """ABMSOD (ellipsoidal Gaussian-weighted windows with bandwidth updates) on the
    PET-like volume: every grid seed x every start radius 4..16, 20 iterations.
    Bound by fp64 arithmetic: the roofline counts the algorithmic fp64 operations
    per window voxel visit (ABM_ALG_OPS_PER_VISIT); the issued fp64 operations
    per visit from the committed counter summary ride along when its sources
    still match (None otherwise)."""
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
    achieved = ABM_ALG_OPS_PER_VISIT * visits_per_s / 1e12
    line["roofline"] = {"bound": "alu", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS, "achieved": achieved,
                        "frac": achieved / FP64_PEAK_TFLOPS, "fp64_ops_per_visit": ABM_ALG_OPS_PER_VISIT,
                        "issued_fp64_ops_per_visit": ops}
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


def _mr_ids(stride):
    """Trajectory ids of every stride-th grid seed of the MR-like workload, all
    scales of each."""
    import oracle
    from paper_1310_6736_amd import synth

    w = synth.mr_blobs()
    S = w.scales[1] - w.scales[0] + 1
    n = oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)
    seeds = np.arange(0, n // S, stride, dtype=np.int64)
    return w, (seeds[:, None] * S + np.arange(S)[None, :]).ravel(), n


def _oracle_shard(job):
    """One worker of the CPU baseline: the oracle on one share of the sample."""
    import oracle

    stride, worker, workers = job
    w, ids, _ = _mr_ids(stride)
    ids = ids[worker::workers]
    _, st = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
    return st["window_evals"], len(ids)


def _pin_one_core():
    cpu = min(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {cpu})


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(stride: int, stride_one: int, workers: int):
    """The oracle as it stands on every stride-th grid seed (all scales) of the
    MR-like workload, sharded over `workers` processes; and on every
    stride_one-th seed in one process pinned to one core.  Window evaluations
    per second of wall time.  Runs before the GPU is initialised (the pools
    fork)."""
    import multiprocessing as mp

    _, ids, n = _mr_ids(stride)
    jobs = [(stride, k, workers) for k in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_shard, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    evals = sum(r[0] for r in res)
    _, ids1, _ = _mr_ids(stride_one)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(1, initializer=_pin_one_core) as pool:
        (e1, _), = pool.map(_oracle_shard, [(stride_one, 0, 1)])
    wall1 = time.perf_counter() - t0
    return {"value": evals / wall, "unit": "window_evals/s", "cores": workers, "kind": "oracle",
            "sample": "every %d-th grid seed x all 21 scales of the MR-like volume (%d of %d trajectories), "
                      "trajectory ids dealt round-robin to %d processes; %.1f s wall" %
                      (stride, ids.size, n, workers, wall),
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "single_core": {"value": e1 / wall1, "unit": "window_evals/s", "cores": 1,
                            "sample": "every %d-th grid seed x all scales (%d trajectories), one process pinned "
                                      "to one core; %.1f s wall" % (stride_one, ids1.size, wall1)}}


def section_only(name, args):
    """One extra section alone, on a fresh context: the workload of a kernel-trace
    profile of that section."""
    stream_ws = stream_workloads(args.serve_requests, max(1, min(16, os.cpu_count() or 1))) \
        if name == "serving" else None
    import torch

    from paper_1310_6736_amd import ks

    ctx = ks.Context(0)
    if name == "serving":
        rec = serving_section(ks, torch, ctx, stream_ws)
    elif name == "batch":
        rec = batch_section(ks, torch, ctx)
    elif name == "pet_like":
        rec = pet_section(ks, torch, ctx, args.steps, args.warmup)
    elif name == "dense_map":
        rec = dense_section(ks, torch, ctx, None)
    elif name == "window_level":
        rec = window_level_section(ks, torch, ctx)
    elif name == "tracking":
        rec = tracking_section(ks, torch, ctx)
    else:
        rec = abmsod_section(ks, torch, ctx, os.path.join(ROOT, "profiles", "alu_k_abmsod_pet128x128x64.json"))
    ctx.close()
    print(json.dumps({"section": name, name: rec}), flush=True)


def timed_steps(ks, torch, ctx, reqs, cap, stream, steps, warmup):
    """Replays of the captured graph of one ks_detect_batch call: warmup untimed,
    then `steps` timed between two device synchronisations.  Profiling is on, so
    each replay's graph also holds event-record nodes around its phases and
    searches; returns (wall seconds, last results, per-step stats)."""
    ks.ks_context_set_profiling(ctx, True)
    try:
        for _ in range(warmup):
            ks.ks_detect_batch(ctx, reqs, capacity=cap, stream=stream)
        torch.cuda.synchronize()
        prof = []
        t0 = time.perf_counter()
        for _ in range(steps):
            res = ks.ks_detect_batch(ctx, reqs, capacity=cap, stream=stream)
            prof.append(ks.ks_last_stats(ctx))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        ks.ks_context_set_profiling(ctx, False)
    return dt, res, prof


def mean_of(prof, key):
    return float(np.mean([p[key] for p in prof]))


def pet_section(ks, torch, ctx, steps, warmup):
    """The PET-like workload: both methods on the 128x128x64 uint16 volume in one
    batched call (the two searches concurrent), the graph replayed; the
    mean-shift search timed inside the step and alone."""
    from paper_1310_6736_amd import synth

    wq, wm = synth.pet_shell(ks.KS_QUADRANT), synth.pet_shell(ks.KS_MEANSHIFT)
    vol = torch.from_numpy(wq.volume).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    cap = 1024
    ks.ks_context_set_profiling(ctx, True)
    iso = {}
    for w in (wq, wm):
        ts = []
        for _ in range(3):
            ks.ks_detect_device(ctx, vol, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap,
                                stream=stream)
            st = ks.ks_last_stats(ctx)
            ts.append(st["ms_search"])
        iso[w.method] = {"stats": st, "search_ms": float(np.median(ts)), "total_ms": st["ms_total"]}
    ks.ks_context_set_profiling(ctx, False)
    reqs = [ks.make_request(vol, w.bins, w.spacing, w.scales, w.method, w.max_iter) for w in (wq, wm)]
    dt, res, prof = timed_steps(ks, torch, ctx, reqs, cap, stream, steps, warmup)
    ms_iso, q_iso = iso[ks.KS_MEANSHIFT]["stats"], iso[ks.KS_QUADRANT]["stats"]
    window_evals = prof[-1]["window_evals"]
    assert window_evals == ms_iso["window_evals"] + q_iso["window_evals"]
    ms_ms, q_ms = mean_of(prof, "ms_search_ms"), mean_of(prof, "ms_search_quad")
    ms_bytes = ms_iso["voxel_visits"] + ms_iso["final_visits"]
    q_bytes = q_iso["voxel_visits"] + q_iso["final_visits"]
    ms_iso_ms, q_iso_ms = iso[ks.KS_MEANSHIFT]["search_ms"], iso[ks.KS_QUADRANT]["search_ms"]
    return {"workload": "PET-like 128x128x64 uint16 ellipsoidal shell, 64 bins, seed spacing 6, scales 4..16, "
                        "max 50 iterations, quadrant + mean-shift in one batched call (the two searches "
                        "concurrent), captured graph replayed",
            "trajectories": {"quadrant": int(q_iso["trajectories"]), "meanshift": int(ms_iso["trajectories"])},
            "value": window_evals / (dt / steps), "unit": "window_evals/s", "ms_per_step": dt * 1e3 / steps,
            "volumes_per_s": steps / dt,
            "regions": {"quadrant": int(res[0][1]), "meanshift": int(res[1][1])},
            "device_ms": {"graph": mean_of(prof, "ms_total"), "search_phase": mean_of(prof, "ms_search"),
                          "quadrant_search": q_ms, "meanshift_search": ms_ms,
                          "prep_ms": mean_of(prof, "ms_prep"), "rank_ms": mean_of(prof, "ms_rank"),
                          "isolated": {"quadrant_search": q_iso_ms, "meanshift_search": ms_iso_ms}},
            "meanshift_search": {"algorithmic_GBs": ms_bytes / (ms_ms * 1e-3) / 1e9,
                                 "algorithmic_GBs_isolated": ms_bytes / (ms_iso_ms * 1e-3) / 1e9,
                                 "swept_GBs_isolated": ms_iso["swept_voxels"] / (ms_iso_ms * 1e-3) / 1e9,
                                 "lds_ops_per_s_isolated": ms_iso["lds_ops"] / (ms_iso_ms * 1e-3)},
            "quadrant_search": {"algorithmic_GBs": q_bytes / (q_ms * 1e-3) / 1e9,
                                "lds_ops_per_s": q_iso["lds_ops"] / (q_ms * 1e-3)}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.section:
        section_only(args.section, args)
        return
    cpu = None
    workers = max(1, min(16, os.cpu_count() or 1))
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample_stride, args.cpu_single_stride, workers)
    stream_ws = None if (args.no_serve or args.main_only) else stream_workloads(args.serve_requests, workers)
    import torch

    from paper_1310_6736_amd import ks, synth

    ctx = ks.Context(0)
    w = synth.mr_blobs()
    vol = torch.from_numpy(w.volume).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    cap = 1024
    req = ks.make_request(vol, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    dt, res, prof = timed_steps(ks, torch, ctx, [req], cap, stream, args.steps, args.warmup)
    st = prof[-1]
    window_evals = int(st["window_evals"])
    assert all(p["window_evals"] == window_evals for p in prof)
    ms_per_step = dt * 1000.0 / args.steps
    k_ms = mean_of(prof, "ms_search_ms")   # the search launch, from the event nodes around it in each replay
    alg = int(st["voxel_visits"] + st["final_visits"])
    swept = int(st["swept_voxels"])
    ops = int(st["lds_ops"])
    achieved = alg / (k_ms * 1e-3) / 1e9
    copy_gbs = ks.ks_roofline(ks.KS_ROOF_COPY) / 1e9
    lds64 = ks.ks_roofline(ks.KS_ROOF_LDS_ADD64)
    traffic = measured_traffic(args.traffic_json)
    issue = measured_record(args.counters_json, "per_launch")
    # host-to-device copy of the input volume (not part of the timed step)
    host = torch.from_numpy(w.volume)
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
        "config": {"workload": "MR-like 256x256x160 int16 (smoothed-noise background, 1-4 heterogeneous blobs), "
                               "64 bins, seed spacing 8, scales 4..24, mean-shift, max 100 iterations; full "
                               "detection (prep, search, ranking of every trajectory, top %d regions to host) as "
                               "one captured-graph replay" % cap,
                   "trajectories": int(st["trajectories"])},
        "volumes_per_s": args.steps / dt,
        "regions": int(res[0][1]),
        "window_evals_per_step": window_evals,
        "device_ms": {"graph": mean_of(prof, "ms_total"), "prep": mean_of(prof, "ms_prep"),
                      "search": k_ms, "rank": mean_of(prof, "ms_rank")},
        # The dominant kernel against three ceilings.  Algorithmic bytes (one byte
        # per window voxel of every evaluation and final pass) are as-if-uncached:
        # they exceed the HBM peak because windows of neighbouring seeds overlap
        # and running-window updates sweep only what changes.  Swept bytes are the
        # voxels the kernel actually reads; LDS atomics its histogram adds.
        "roofline": {"bound": "hbm", "kernel": "k_search_ms", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "device_ms": k_ms, "algorithmic_bytes_per_launch": alg,
                     "swept": {"bytes_per_launch": swept, "achieved": swept / (k_ms * 1e-3) / 1e9,
                               "frac": swept / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
                     "lds_atomic": {"ops_per_launch": ops, "achieved": ops / (k_ms * 1e-3), "peak": lds64,
                                    "unit": "lane-ops/s", "peak_kind": "conflict-free 64-bit LDS add microbenchmark",
                                    "frac": ops / (k_ms * 1e-3) / lds64},
                     "copy_peak_measured": copy_gbs,
                     "binding": issue},
        "h2d": dict(h2d, bytes=int(w.volume.nbytes),
                    pcie_inclusive_window_evals_per_s=window_evals / (dt / args.steps + h2d["pinned_ms"] * 1e-3)),
    }
    if not args.main_only:
        line["pet_like"] = pet_section(ks, torch, ctx, args.steps, args.warmup)
        line["dense_map"] = dense_section(ks, torch, ctx, None)
        line["window_level"] = window_level_section(ks, torch, ctx)
        line["tracking"] = tracking_section(ks, torch, ctx)
        line["abmsod"] = abmsod_section(ks, torch, ctx, args.abmsod_ops_json)
    if not (args.no_batch or args.main_only):
        line["batch"] = batch_section(ks, torch, ctx)
    if not (args.no_serve or args.main_only):
        line["serving"] = serving_section(ks, torch, ctx, stream_ws)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
