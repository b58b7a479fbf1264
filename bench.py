#!/usr/bin/env python3
"""Benchmark: seed-scale window evaluations per second on the PET-like workload.

One step = one full detection pass over the resident 128x128x64 uint16 PET-like
volume (64 bins, seed spacing 6, scales 4..16, 50 iterations) with both methods:
quadrant ascent and mean-shift toward the uniform pmf (range scan, binning,
persistent searches with the final saliency pass, device ranking, results to
host).  The input is in HBM before the timed region starts.

Prints one JSON line.  Extra fields: volumes/s, per-method device times, the
roofline of the dominant kernel (the mean-shift search) measured with HIP events
on the launch stream, and the CPU oracle timed on a bounded sample.  Optional
--serve adds a Poisson serving run against a plain one-launch-per-volume loop.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-stride", type=int, default=2)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_meanshift_pet.json"))
    return ap.parse_args()


def cpu_baseline(stride: int):
    """The oracle as it stands, single-threaded, on every stride-th trajectory of the
    same workload; window evaluations per second."""
    import oracle
    from paper_1310_6736_amd import synth

    total_evals, total_s = 0, 0.0
    sample = []
    for method in (0, 1):
        w = synth.pet_shell(method)
        n = oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)
        ids = np.arange(0, n, stride, dtype=np.int64)
        t0 = time.perf_counter()
        _, st = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
        total_s += time.perf_counter() - t0
        total_evals += st["window_evals"]
        sample.append(f"{w.name}: {len(ids)}/{n} trajectories")
    return {"value": total_evals / total_s, "unit": "window_evals/s", "cores": 1, "kind": "oracle",
            "sample": "every %dth trajectory of the PET-like volume, both methods (%s); %.1f s" %
                      (stride, "; ".join(sample), total_s)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1310_6736_amd import ks, synth

    dev = torch.device("cuda:0")
    ctx = ks.Context(0)
    wq = synth.pet_shell(ks.KS_QUADRANT)
    wm = synth.pet_shell(ks.KS_MEANSHIFT)
    vol = torch.from_numpy(wq.volume).to(dev)
    stream = torch.cuda.current_stream()
    cap = 1024

    def step(profile_sink=None):
        out = []
        for w in (wq, wm):
            regs, n = ks.ks_detect_device(ctx, vol, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                          capacity=cap, stream=stream)
            st = ks.ks_last_stats(ctx)
            if profile_sink is not None:
                profile_sink.append((w.method, st))
            out.append((n, st))
        return out

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

    window_evals = sum(st["window_evals"] for _, st in res)
    ms_per_step = dt * 1000.0 / args.steps
    ms_stats = [st for m, st in prof if m == ks.KS_MEANSHIFT]
    q_stats = [st for m, st in prof if m == ks.KS_QUADRANT]
    ms_kernel_ms = float(np.mean([s["ms_search"] for s in ms_stats]))
    q_kernel_ms = float(np.mean([s["ms_search"] for s in q_stats]))
    ms_bytes = ms_stats[-1]["voxel_visits"] + ms_stats[-1]["final_visits"]
    q_bytes = q_stats[-1]["voxel_visits"] + q_stats[-1]["final_visits"]
    achieved = ms_bytes / (ms_kernel_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            traffic = json.load(open(args.traffic_json)).get("bytes_per_launch")
        except Exception:
            traffic = None

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
                               "scales 4..16, max 50 iterations, quadrant + mean-shift",
                   "trajectories": {"quadrant": int(res[0][1]["trajectories"]),
                                    "meanshift": int(res[1][1]["trajectories"])}},
        "volumes_per_s": 1000.0 / ms_per_step,
        "regions": {"quadrant": int(res[0][0]), "meanshift": int(res[1][0])},
        "window_evals_per_step": int(window_evals),
        "device_ms": {"quadrant_search": q_kernel_ms, "meanshift_search": ms_kernel_ms,
                      "prep_ms": float(np.mean([s["ms_prep"] for _, s in prof])),
                      "rank_ms": float(np.mean([s["ms_rank"] for _, s in prof]))},
        "roofline": {"bound": "hbm", "kernel": "k_search_ms", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": int(ms_bytes),
                     "quadrant_achieved": q_bytes / (q_kernel_ms * 1e-3) / 1e9},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_stride)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
