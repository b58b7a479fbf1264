"""GPU tests of the batched launch (one captured graph over many volumes) and of
the continuous-batching server: every volume's result must equal the same
volume run alone (bit-identical regions) and, on a subset, the CPU oracle."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1310_6736_amd import ks, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    c = ks.Context(0)
    yield c
    c.close()


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def small_mix():
    """Eight volumes of uneven sizes and all three voxel types, both methods,
    several bin counts and scale ranges."""
    dims = [(40, 33, 29), (37, 52, 31), (64, 48, 33), (45, 45, 45), (70, 35, 40), (33, 61, 37), (50, 50, 34),
            (66, 41, 43)]
    dtypes = [np.uint8, np.uint16, np.int16]
    out = []
    for i, (X, Y, Z) in enumerate(dims):
        rng = np.random.default_rng(500 + i)
        dt = dtypes[i % 3]
        hi = 255 if dt == np.uint8 else 3000
        v = np.clip(rng.normal(hi * 0.2, hi * 0.03, (Z, Y, X)), 0, hi)
        zz, yy, xx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
        for _ in range(2):
            r = int(rng.integers(4, 9))
            c = [int(rng.integers(r, d - r)) for d in (X, Y, Z)]
            m = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
            v[m] = rng.integers(0, hi + 1, int(m.sum()))
        vol = np.rint(v).astype(dt)
        bins = [32, 64, 48][i % 3]
        scales = [(3, 8), (2, 7), (4, 10)][i % 3]
        out.append(synth.Workload(f"mix{i}", vol, bins, 5 + i % 3, scales, i % 2, 30))
    return out


def same_regions(a, b):
    return a[1] == b[1] and np.array_equal(a[0], b[0])


RTOL = 1e-5


def close32(got, want):
    """float32 reported values within 1e-5 relative of the oracle's doubles, and
    exactly zero where those are zero."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    ok = np.abs(got - want) <= RTOL * np.abs(want)
    return bool(np.all(np.where(want == 0.0, got == 0.0, ok)))


def assert_matches_oracle(got, n_got, want, n_want, label):
    assert n_got == n_want, (label, n_got, n_want)
    assert len(got) == len(want), label
    for f in ("x", "y", "z", "scale", "seed"):
        assert np.array_equal(got[f], want[f]), (label, f)
    for f in ("saliency", "entropy", "pdf_change"):
        assert close32(got[f], want[f]), (label, f)


def test_batch_equals_alone_and_oracle(torch_dev, ctx):
    ws = small_mix()
    note(f"batch of {len(ws)} small volumes")
    vols = [torch_dev.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    cap = 4096
    batch = ks.ks_detect_batch(ctx, reqs, capacity=cap)
    for i, (w, v) in enumerate(zip(ws, vols)):
        alone = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
        assert same_regions(batch[i], alone), i
        want, n_want, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
        assert_matches_oracle(batch[i][0], batch[i][1], want, n_want, i)


def test_batch_graph_replays_are_stable(torch_dev, ctx):
    ws = small_mix()[:5]
    note("batch graph replay x3 with eager work between")
    vols = [torch_dev.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    first = ks.ks_detect_batch(ctx, reqs, capacity=512)
    for _ in range(3):
        # unrelated eager work on the same context between replays
        ks.ks_detect_device(ctx, vols[0], 16, 5, (2, 4), ks.KS_MEANSHIFT, 5, capacity=8)
        again = ks.ks_detect_batch(ctx, reqs, capacity=512)
        for a, b in zip(first, again):
            assert same_regions(a, b)


def test_batch_of_64_uneven_volumes(torch_dev, ctx):
    """The uneven 64-volume batch: each result equals the volume run alone; the
    oracle checks every sphere-type volume and the two smallest of each other type."""
    specs = synth.batch_specs()
    note("generating the 64-volume batch")
    ws = synth.batch_workloads()
    vols = [torch_dev.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    note("batch of 64")
    batch = ks.ks_detect_batch(ctx, reqs, capacity=256)
    def size(i):
        return specs[i][1][0] * specs[i][1][1] * specs[i][1][2]

    oracle_ids = [i for i, s in enumerate(specs) if s[0] == 0]
    for kind in (1, 2):
        oracle_ids += sorted((i for i, s in enumerate(specs) if s[0] == kind), key=size)[:2]
    for i, (w, v) in enumerate(zip(ws, vols)):
        alone = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=256)
        assert same_regions(batch[i], alone), i
    for i in oracle_ids:
        w = ws[i]
        note(f"oracle on batch volume {i} ({w.name})")
        want, n_want, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=256)
        assert_matches_oracle(batch[i][0], batch[i][1], want, n_want, i)


def test_batch_without_stream_waits_for_the_volume_writes(torch_dev, ctx):
    """A batch called without a stream runs on the context's own stream, after
    the work queued on the null stream before the call: here a chain of matrix
    products and then the copy that writes the volume."""
    w = small_mix()[3]
    note("batch without a stream after a device write of its volume")
    src = torch_dev.from_numpy(w.volume).to("cuda:0")
    alone = ks.ks_detect_device(ctx, src, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
    torch_dev.cuda.synchronize()
    for rep in range(2):
        t = torch_dev.zeros_like(src)
        a = torch_dev.ones((2048, 2048), dtype=torch_dev.float32, device="cuda:0")
        torch_dev.cuda.synchronize()
        for _ in range(6):   # several milliseconds of queued work before the write
            a = (a @ a) * (1.0 / 2048.0)
        t.copy_(src)
        got = ks.ks_detect_batch(ctx, [ks.make_request(t, w.bins, w.spacing, w.scales, w.method, w.max_iter)],
                                 capacity=4096)[0]
        assert same_regions(got, alone), rep
    torch_dev.cuda.synchronize()


def test_server_results_equal_alone(torch_dev, ctx):
    ws = small_mix()
    note("server: 16 requests, 4 slots")
    srv = ks.Server(0, hbm_budget=2 << 30, max_slots=4)
    try:
        tickets = []
        for rep in range(2):
            for w in ws:
                tickets.append((w, srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter)))
                time.sleep(0.002)
        srv.drain()
        for w, t in tickets:
            got = srv.poll(t, capacity=4096)
            assert got is not None
            v = torch_dev.from_numpy(w.volume).to("cuda:0")
            alone = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
            assert same_regions(got, alone), w.name
        st = srv.stats()
        assert st["completed"] == len(tickets) and st["p99_ms"] >= st["p50_ms"] > 0
        # a new measurement window counts only what is submitted after it
        srv.reset_stats()
        st = srv.stats()
        assert st["completed"] == 0 and st["submitted"] == 0 and st["p50_ms"] == 0 and st["volumes_per_s"] == 0
        t2 = [srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter) for w in ws[:2]]
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 2 and st["submitted"] == 2 and st["volumes_per_s"] > 0
        for w, t in zip(ws[:2], t2):
            v = torch_dev.from_numpy(w.volume).to("cuda:0")
            alone = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
            assert same_regions(srv.poll(t, capacity=4096), alone), w.name
    finally:
        srv.close()


def test_server_small_budget_queues_and_refuses(torch_dev, ctx):
    ws = small_mix()[:4]
    note("server: small budget")
    one = 3 << 20
    srv = ks.Server(0, hbm_budget=one, max_slots=2)
    try:
        with pytest.raises(ks.KsError) as e:
            srv.submit(synth.spheres_64().volume, 32, 2, (3, 8), ks.KS_MEANSHIFT, 10)
        assert e.value.status == ks.KS_E_TOO_LARGE
        ts = [srv.submit(x.volume, x.bins, x.spacing, x.scales, x.method, x.max_iter) for x in ws]
        srv.drain()
        for x, t in zip(ws, ts):
            got = srv.poll(t, capacity=1024)
            v = torch_dev.from_numpy(x.volume).to("cuda:0")
            alone = ks.ks_detect_device(ctx, v, x.bins, x.spacing, x.scales, x.method, x.max_iter, capacity=1024)
            assert same_regions(got, alone)
        assert srv.stats()["refused"] == 1
    finally:
        srv.close()


def test_server_budget_bounds_the_device_memory_of_its_slots(torch_dev, ctx):
    """A large request (the PET-like volume, mean-shift: about 15 MB of device
    memory alone), then many small ones that run on the other slots while it
    does, then the large one again: the bytes the slots hold never exceed the
    budget (idle slots give back what a new batch would not fit beside), and
    every result equals the volume run alone."""
    big = synth.pet_shell(ks.KS_MEANSHIFT)
    ws = [big] + small_mix() * 3 + [big]
    budget = 24 << 20
    note("server: device memory of the slots within the budget")
    srv = ks.Server(0, hbm_budget=budget, max_slots=4)
    try:
        tickets = [(w, srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter)) for w in ws]
        srv.drain()
        st = srv.stats()
        got = [(w, srv.poll(t, capacity=100000)) for w, t in tickets]
    finally:
        srv.close()
    assert st["refused"] == 0 and st["completed"] == len(ws)
    assert 0 < st["bytes_peak"] <= budget, st
    assert st["bytes_in_use"] <= budget, st
    alone = {}
    for w, res in got:
        if w.name not in alone:
            v = torch_dev.from_numpy(w.volume).to("cuda:0")
            alone[w.name] = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                                capacity=100000)
        assert same_regions(res, alone[w.name]), w.name


def test_server_large_request_among_small_ones(torch_dev, ctx):
    """An MR-like request (large: run alone, its search in several launches)
    submitted between small ones, and a second one right after it: every result
    equals the volume run alone."""
    big = synth.mr_blobs()
    ws = small_mix()[:3] + [big] + small_mix()[3:6] + [big] + small_mix()[6:]
    note("server: large requests among small ones")
    srv = ks.Server(0, hbm_budget=4 << 30, max_slots=4)
    try:
        # the second large request keeps only its top 100 regions
        tickets = [(w, i, srv.submit(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                     max_regions=100 if i == 7 else 0)) for i, w in enumerate(ws)]
        srv.drain()
        got = [(w, i, srv.poll(t, capacity=4096)) for w, i, t in tickets]
    finally:
        srv.close()
    alone = {}
    for w, i, res in got:
        if w.name not in alone:
            v = torch_dev.from_numpy(w.volume).to("cuda:0")
            alone[w.name] = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                                capacity=4096)
        if i == 7:
            # the total found, and the top 100 in rank order
            assert res[1] == alone[w.name][1] and np.array_equal(res[0], alone[w.name][0][:100]), w.name
        else:
            assert same_regions(res, alone[w.name]), w.name


def moving_frames(n, seed, shape=(36, 40, 44)):
    """A textured sphere in noise moving 2 voxels per frame along x and 1 along y."""
    Z, Y, X = shape
    rng = np.random.default_rng(seed)
    zz, yy, xx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    frames = []
    for f in range(n):
        v = np.clip(np.rint(rng.normal(50, 4, shape)), 0, 255).astype(np.uint8)
        c = (12 + 2 * f, 14 + f, 18)
        m = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= 36
        v[m] = rng.integers(0, 256, int(m.sum()))
        frames.append(v)
    return frames


def handed_over(regions, max_seeds):
    """Start positions of the next frame: the first max_seeds distinct positions
    of the frame's regions in rank order."""
    out = []
    for r in regions:
        p = (int(r["x"]), int(r["y"]), int(r["z"]))
        if p not in out:
            out.append(p)
        if len(out) == max_seeds:
            break
    return out


def test_server_tracked_frames_start_from_the_previous_regions(torch_dev):
    frames = moving_frames(4, 900)
    bins, sp, max_iter, max_seeds = 32, 6, 30, 6
    tracks = {7: (ks.KS_QUADRANT, (3, 7)), 8: (ks.KS_MEANSHIFT, (3, 6))}
    note("server: two tracked sequences and untracked requests")
    srv = ks.Server(0, hbm_budget=1 << 30, max_slots=4)
    try:
        tickets = []
        for f, v in enumerate(frames):
            for tid, (method, scales) in tracks.items():
                t = srv.submit(v, bins, sp, scales, method, max_iter, track=tid, max_seeds=max_seeds)
                tickets.append((tid, f, t))
            tickets.append((None, f, srv.submit(v, bins, sp, (3, 7), ks.KS_QUADRANT, max_iter)))
        srv.drain()
        got = {(tid, f): srv.poll(t, capacity=100000) for tid, f, t in tickets}
    finally:
        srv.close()
    for tid, (method, scales) in list(tracks.items()) + [(None, (ks.KS_QUADRANT, (3, 7)))]:
        seeds = None
        for f, v in enumerate(frames):
            want, wn, _ = oracle.detect(v, bins, sp, scales, method, max_iter, seeds=seeds)
            regs, n = got[(tid, f)]
            assert n == wn, (tid, f)
            for fld in ("x", "y", "z", "scale", "seed"):
                assert np.array_equal(regs[fld], want[fld]), (tid, f, fld)
            assert np.allclose(regs["saliency"], want["saliency"], rtol=1e-5, atol=0), (tid, f)
            if tid is not None:
                nxt = handed_over(want, max_seeds)
                seeds = nxt if nxt else None
    # a warm-started frame runs max_seeds trajectories per scale, not the grid
    assert got[(7, 3)][1] <= max_seeds


def test_batch_overlapped_searches_equal_sequential(torch_dev, ctx):
    """The quadrant and mean-shift searches of a batch run concurrently on two
    streams by default; results equal the sequential launch order, through the
    captured graph and through the direct (profiled) launch sequence."""
    ws = small_mix()
    vols = [torch_dev.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    note("batch: overlapped vs sequential searches")
    out = {}
    try:
        for ov in (0, 1):
            ks.ks_context_set_overlap(ctx, ov)
            for prof in (0, 1):
                ks.ks_context_set_profiling(ctx, prof)
                out[(ov, prof)] = ks.ks_detect_batch(ctx, reqs, capacity=4096)
                if prof:
                    st = ks.ks_last_stats(ctx)
                    assert st["ms_search_quad"] > 0 and st["ms_search_ms"] > 0
    finally:
        ks.ks_context_set_overlap(ctx, 1)
        ks.ks_context_set_profiling(ctx, 0)
    ref = out[(0, 0)]
    for key, res in out.items():
        for i in range(len(ws)):
            assert res[i][1] == ref[i][1] and np.array_equal(res[i][0], ref[i][0]), (key, i)


def test_batch_window_levels_and_scale_groups_match_oracle(torch_dev, ctx):
    """Mean-shift volumes with and without window levels, different bin counts
    and scale ranges in one batch, scale groups forced to 3 (groups cross the
    replica change at s = 6 -> 7, and a wave moves between volumes' layouts):
    every volume equals the oracle."""
    specs = [("w32", np.uint16, (22, 25, 28), 32, (4, 9), (900, 2100)),
             ("w64", np.int16, (20, 23, 26), 64, (3, 10), (-300, 600)),
             ("full", np.uint16, (21, 24, 27), 48, (5, 8), None)]
    vols, reqs = [], []
    for i, (name, dt, shape, bins, scales, win) in enumerate(specs):
        rng = np.random.default_rng(700 + i)
        lo, hi = (-900, 2000) if dt == np.int16 else (0, 3000)
        v = rng.integers(lo, hi + 1, shape).astype(dt)
        vols.append(v)
        t = torch_dev.from_numpy(v).to("cuda:0")
        reqs.append(ks.make_request(t, bins, 4, scales, ks.KS_MEANSHIFT, 20,
                                    opts=ks.options(window=win) if win else None))
        reqs[-1]._keep = t
    note("batch: window levels with scale groups")
    ks.ks_context_set_ms_group(ctx, 3)
    try:
        out = ks.ks_detect_batch(ctx, reqs, capacity=100000)
    finally:
        ks.ks_context_set_ms_group(ctx, 0)
    for (name, dt, shape, bins, scales, win), v, (got, n) in zip(specs, vols, out):
        want, n_want, _ = oracle.detect(v, bins, 4, scales, ks.KS_MEANSHIFT, 20, capacity=100000, window=win)
        assert n == n_want, name
        for f in ("x", "y", "z", "scale", "seed"):
            assert np.array_equal(got[f], want[f]), (name, f)
        assert np.allclose(got["saliency"], want["saliency"], rtol=1e-5, atol=0), name


def test_batch_autotune_keeps_results(torch_dev):
    """The batch autotuner picks shapes within their ranges, and the batch run
    with them equals the batch with the default shapes."""
    ws = small_mix()
    vols = [torch_dev.from_numpy(w.volume).to("cuda:0") for w in ws]
    reqs = [ks.make_request(v, w.bins, w.spacing, w.scales, w.method, w.max_iter) for v, w in zip(vols, ws)]
    note("batch autotune")
    base_ctx = ks.Context(0)
    ctx = ks.Context(0)
    try:
        base = ks.ks_detect_batch(base_ctx, reqs, capacity=4096)
        t = ks.ks_context_autotune_batch(ctx, reqs, reps=1)
        assert 3 <= t[0] <= 5 and 2 <= t[1] <= 3 and t[2] in (4, 6, 8) and 0 <= t[3] <= 2 and 0 <= t[4] <= 4, t
        got = ks.ks_detect_batch(ctx, reqs, capacity=4096)
        for i, (a, b) in enumerate(zip(base, got)):
            assert same_regions(a, b), i
        with pytest.raises(ks.KsError):
            ks.ks_context_autotune_batch(ctx, reqs, reps=0)
    finally:
        ctx.close()
        base_ctx.close()
