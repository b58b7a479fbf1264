"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer results (bins, histograms, positions, iterations, stop reasons, scales,
kept flags, seeds, region order) must be bit-identical; the double-precision
decision values (objective, saliency used for ranking) must be equal; the
float32 reported entropy / pdf change / saliency must be within 1e-5 relative of
the oracle's accurate double values, and exactly zero where those are zero.
"""
import ctypes
import os
import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_1310_6736_amd import ks, synth

pytestmark = pytest.mark.gpu

RTOL = 1e-5


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


def restore_tuning(ctx):
    """The context's default tuning (4 / 1 replicas, 4 replicas up to s = 6)."""
    ks.ks_context_set_tuning(ctx, 4, 0)
    ks.ks_context_set_tuning_small(ctx, 2, 6)


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(torch, vol):
    return torch.from_numpy(np.ascontiguousarray(vol)).to("cuda:0")


def close32(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    zero = want == 0.0
    ok = np.abs(got - want) <= RTOL * np.abs(want)
    return bool(np.all(np.where(zero, got == 0.0, ok)))


def random_volume(seed, shape, dtype, lo, hi):
    rng = np.random.default_rng(seed)
    v = rng.integers(lo, hi + 1, shape).astype(dtype)
    # a smoother low-entropy region and a textured block, for skewed histograms
    z, y, x = shape
    v[: z // 2, : y // 2, :] = (lo + (hi - lo) // 3)
    v[z // 3: z // 3 + 5, y // 4: y // 4 + 6, x // 5: x // 5 + 7] = rng.integers(lo, hi + 1, (min(5, z - z // 3),
                                                                                               min(6, y - y // 4),
                                                                                               min(7, x - x // 5)))
    return v


# ------------------------------------------------------------------ binning

@pytest.mark.parametrize("case", [
    ("u8", np.uint8, (13, 17, 23), 0, 255, 32),
    ("u16", np.uint16, (9, 31, 37), 0, 4095, 64),
    ("i16", np.int16, (11, 7, 65), -900, 1400, 7),
    ("i16full", np.int16, (4, 8, 17), -32768, 32767, 256),
    ("u8narrow", np.uint8, (5, 6, 19), 17, 23, 64),
])
def test_bin_volume_bit_exact(torch_dev, ctx, case):
    name, dt, shape, lo, hi, bins = case
    note(f"bin_volume {name} {shape} B={bins}")
    v = random_volume(1, shape, dt, lo, hi)
    got = ks.ks_bin_volume(ctx, dev(torch_dev, v), bins)
    assert np.array_equal(got, oracle.bin_volume(v, bins))


@pytest.mark.parametrize("case", [
    ("u8", np.uint8, (13, 17, 23), 0, 255, 32),
    ("u16", np.uint16, (9, 31, 37), 0, 4095, 64),
    ("i16", np.int16, (11, 7, 65), -900, 1400, 7),
])
def test_bin_volume_unaligned_volume(torch_dev, ctx, case):
    """A volume that starts one element into its allocation (not 16-byte aligned:
    the range scan takes its voxel-by-voxel path), and one that starts 16 bytes in."""
    name, dt, shape, lo, hi, bins = case
    v = random_volume(2, shape, dt, lo, hi)
    want = oracle.bin_volume(v, bins)
    flat = np.ascontiguousarray(v).reshape(-1)
    esize = np.dtype(dt).itemsize
    for skip in (1, 16 // esize):
        note(f"bin_volume {name} {shape} B={bins}, {skip} element(s) into the buffer")
        # bytes placed in a uint8 buffer, then viewed as the voxel type
        off = skip * esize
        buf = torch_dev.zeros(flat.nbytes + 64, dtype=torch_dev.uint8, device="cuda:0")
        buf[off:off + flat.nbytes] = torch_dev.from_numpy(flat.view(np.uint8)).to("cuda:0")
        view = buf[off:off + flat.nbytes].view(dev(torch_dev, flat[:1]).dtype).view(*shape)
        assert view.is_contiguous() and (view.data_ptr() % 16 != 0) == (skip * esize % 16 != 0)
        got = ks.ks_bin_volume(ctx, view, bins)
        assert np.array_equal(got, want), (name, skip)


def test_bin_volume_full_size_workloads(torch_dev, ctx):
    for w in (synth.pet_shell(ks.KS_QUADRANT), synth.mr_blobs()):
        note(f"bin_volume {w.name}")
        got = ks.ks_bin_volume(ctx, dev(torch_dev, w.volume), w.bins)
        assert np.array_equal(got, oracle.bin_volume(w.volume, w.bins))


# --------------------------------------------------------------- histograms

def positions(shape, n, seed):
    z, y, x = shape
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (x - 1, y - 1, z - 1), (x - 1, 0, z // 2), (x // 2, y // 2, z // 2), (1, y - 2, 3 % z)]
    pts += [tuple(int(a) for a in rng.integers(0, (x, y, z))) for _ in range(n)]
    return np.array(pts, np.int32)


@pytest.mark.parametrize("bins", [2, 32, 64, 100, 256])
@pytest.mark.parametrize("rl", [6, 4, 2])
def test_meanshift_window_stats_bit_exact(torch_dev, ctx, bins, rl):
    note(f"hist meanshift B={bins} rl={rl}")
    v = random_volume(bins + rl, (37, 41, 45), np.uint16, 0, 4095)
    bv = oracle.bin_volume(v, bins)
    pts = positions(v.shape, 20, 7)
    rng = np.random.default_rng(3)
    sc = rng.integers(1, 33, len(pts)).astype(np.int32)
    sc[:3] = [32, 1, 16]
    ks.ks_context_set_tuning(ctx, rl, 3)
    try:
        got = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_MEANSHIFT, pts, sc)
        cube = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_CUBE, pts, sc)
    finally:
        restore_tuning(ctx)
    for i, p in enumerate(pts):
        counts, msum, _, _ = oracle.eval_meanshift(bv, bins, p, int(sc[i]))
        assert np.array_equal(got[i, 0], counts.astype(np.int32)), (i, p, sc[i])
        assert np.array_equal(got[i, 1:].T, msum.astype(np.int32)), (i, p, sc[i])
        assert np.array_equal(cube[i], counts), (i, p, sc[i])


def move_pairs(shape, seed):
    """(P, Q, s) triples for the running-window update: small moves in every
    direction, zero moves, moves across the volume border, moves longer than the
    window, both corners, and the largest scale."""
    z, y, x = shape
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(40):
        s = int(rng.integers(1, 33))
        p = [int(a) for a in rng.integers(0, (x, y, z))]
        d = [int(a) for a in rng.integers(-s, s + 1, 3)]
        q = [min(max(p[a] + d[a], 0), (x, y, z)[a] - 1) for a in range(3)]
        out.append((p, q, s))
    out += [([0, 0, 0], [1, 1, 1], 3), ([x - 1, y - 1, z - 1], [x - 2, y - 1, z - 3], 5),
            ([5, 6, 7], [5, 6, 7], 4), ([0, y // 2, z // 2], [x - 1, y // 2, z // 2], 2),
            ([x // 2, y // 2, z // 2], [x // 2 + 1, y // 2 - 2, z // 2], 32), ([3, 3, 3], [3, 3, 4], 1),
            ([x // 2, 2, z - 2], [x // 2 - 9, 0, z - 1], 9)]
    return out


@pytest.mark.parametrize("bins", [2, 64, 256])
@pytest.mark.parametrize("rl", [2, 4, 6])
def test_meanshift_running_window_update_bit_exact(torch_dev, ctx, bins, rl):
    """A window updated from P to Q (voxels leaving taken out, offsets shifted,
    voxels entering added) equals the oracle's fresh window at Q."""
    note(f"hist ms move B={bins} rl={rl}")
    v = random_volume(bins * 3 + rl, (37, 41, 45), np.uint16, 0, 4095)
    bv = oracle.bin_volume(v, bins)
    trip = move_pairs(v.shape, bins + rl)
    pq = np.array([p + q for p, q, _ in trip], np.int32)
    sc = np.array([s for _, _, s in trip], np.int32)
    ks.ks_context_set_tuning(ctx, rl, 0)
    try:
        got = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_MS_MOVE, pq, sc)
    finally:
        restore_tuning(ctx)
    for i, (p, q, s) in enumerate(trip):
        counts, msum, _, _ = oracle.eval_meanshift(bv, bins, q, s)
        assert np.array_equal(got[i, 0], counts.astype(np.int32)), (i, p, q, s)
        assert np.array_equal(got[i, 1:].T, msum.astype(np.int32)), (i, p, q, s)


@pytest.mark.parametrize("bins", [2, 64, 256])
def test_meanshift_inner_cube_counts_bit_exact(torch_dev, ctx, bins):
    """The final pass's inner-cube counts, through the shell subtraction and swept
    directly, equal the oracle's cube of half-width s-1 (s = 1: one voxel)."""
    note(f"hist ms inner B={bins}")
    v = random_volume(bins + 11, (29, 33, 47), np.uint8, 0, 255)
    bv = oracle.bin_volume(v, bins)
    pts = positions(v.shape, 20, 9)
    rng = np.random.default_rng(bins)
    sc = rng.integers(1, 33, len(pts)).astype(np.int32)
    sc[:4] = [1, 32, 2, 1]
    got = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_MS_INNER, pts, sc)
    for i, p in enumerate(pts):
        s = int(sc[i])
        assert np.array_equal(got[i, 0], oracle.hist_cube(bv, bins, p, s)), (i, p, s)
        inner = oracle.hist_cube(bv, bins, p, s - 1)
        assert np.array_equal(got[i, 1], inner), (i, p, s, "shell")
        assert np.array_equal(got[i, 2], inner), (i, p, s, "inner")


@pytest.mark.parametrize("bins,rng_", [(32, (3, 8)), (64, (4, 16)), (256, (1, 5)), (13, (2, 2)), (64, (1, 32))])
@pytest.mark.parametrize("rq", [3, 0])
def test_octant_histograms_bit_exact(torch_dev, ctx, bins, rng_, rq):
    note(f"hist octants B={bins} range={rng_} rq={rq}")
    v = random_volume(5, (30, 33, 71), np.uint8, 0, 255)
    bv = oracle.bin_volume(v, bins)
    pts = positions(v.shape, 6, 11)
    ks.ks_context_set_tuning(ctx, 6, rq)
    try:
        got = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_OCTANTS, pts, scale_range=rng_)
    finally:
        restore_tuning(ctx)
    for i, p in enumerate(pts):
        for j in range(8):
            for kk, k in enumerate(range(rng_[0], rng_[1] + 1)):
                assert np.array_equal(got[i, j, kk], oracle.hist_octant(bv, bins, p, j, k)), (i, j, k)


@pytest.mark.parametrize("bins,rng_", [(32, (2, 9)), (64, (3, 17)), (256, (0, 4)), (64, (0, 33))])
def test_centred_shell_histograms_bit_exact(torch_dev, ctx, bins, rng_):
    note(f"hist shells B={bins} range={rng_}")
    v = random_volume(6, (40, 29, 50), np.int16, -300, 2000)
    bv = oracle.bin_volume(v, bins)
    pts = positions(v.shape, 6, 12)
    got = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_SHELLS, pts, scale_range=rng_)
    for i, p in enumerate(pts):
        for kk, s in enumerate(range(rng_[0], rng_[1] + 1)):
            assert np.array_equal(got[i, kk], oracle.hist_cube(bv, bins, p, s)), (i, s)


# -------------------------------------------------------------- trajectories

def compare_traces(got, want, label):
    assert len(got) == len(want), label
    for f in ("x0", "y0", "z0", "x", "y", "z", "scale", "iters", "stop", "keep"):
        bad = np.nonzero(got[f] != want[f])[0]
        assert bad.size == 0, f"{label}: {f} differs at {bad[:10]} got {got[f][bad[:5]]} want {want[f][bad[:5]]}"
    assert np.array_equal(got["objective"], want["objective"]), label
    assert np.array_equal(got["saliency64"], want["y64"]), label
    keep = want["keep"] == 1
    assert close32(got["entropy"][keep], want["h_ref"][keep]), label
    assert close32(got["pdf_change"][keep], want["w64"][keep]), label
    assert close32(got["saliency"][keep], want["y_ref"][keep]), label


def test_traces_spheres64_quadrant(torch_dev, ctx):
    w = synth.spheres_64()
    note(f"traces {w.name}")
    got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    want, _ = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    compare_traces(got, want, w.name)


@pytest.mark.parametrize("method", [ks.KS_QUADRANT, ks.KS_MEANSHIFT])
def test_traces_pet_shell_full(torch_dev, ctx, method):
    w = synth.pet_shell(method)
    note(f"traces {w.name}")
    got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    want, _ = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    compare_traces(got, want, w.name)


@pytest.mark.parametrize("update", [0, 200], ids=["fresh", "always"])
def test_traces_meanshift_update_settings(torch_dev, ctx, update):
    """Mean-shift traces are the same with running-window updates off (every
    evaluation sweeps its whole window) and with updates taken wherever the two
    difference regions are smaller than twice the window."""
    w = synth.pet_shell(ks.KS_MEANSHIFT)
    note(f"traces {w.name} update={update}")
    ks.ks_context_set_ms_update(ctx, update)
    try:
        got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    finally:
        ks.ks_context_set_ms_update(ctx, 100)
    ids = np.arange(0, len(got), 5)
    want, _ = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
    compare_traces(got[ids], want, f"{w.name} update={update}")


def mr_oracle_run():
    """The oracle's run of every MR-like trajectory, computed by the host pool
    that started at collection."""
    import oracle_pool

    if not oracle_pool.started():
        pytest.skip("the oracle pool did not start (no GPU device node at collection)")
    arr, st, wall = oracle_pool.result()
    note(f"oracle pool: {len(arr)} trajectories in {wall:.1f} s on {oracle_pool.workers()} processes")
    return arr, st


def test_traces_mr_blobs_full(torch_dev, ctx):
    """Every one of the 430,080 mean-shift trajectories of the MR-like volume (256 x
    256 x 160 int16, 64 bins, spacing 8, scales 4..24, 100 iterations) against the
    oracle: positions, iterations, stop reasons, scales, kept flags, the double
    objective and saliency bit-identical, float32 values within 1e-5."""
    w = synth.mr_blobs()
    note(f"traces {w.name} (full GPU run, full oracle run)")
    got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    want, _ = mr_oracle_run()
    compare_traces(got, want, w.name)


def test_detect_mr_blobs_full_matches_oracle(torch_dev, ctx):
    """The ranked detection of the MR-like volume at full size (343,194 regions from
    430,080 trajectories: the compaction, the 524,288-record sort and the dedup at
    their largest tested size) against the oracle's ranking of its own full run:
    positions, scales and seeds bit-identical in rank order, float32 saliency,
    entropy and pdf change within 1e-5 with exact zeros; then the top 1,000 alone,
    the work counters against the oracle's, and the same volume through a batch
    request and the captured graph."""
    w = synth.mr_blobs()
    note(f"detect {w.name} full")
    t = dev(torch_dev, w.volume)
    n_traj = oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)
    got, n = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=n_traj)
    st = ks.ks_last_stats(ctx)
    traj, ost = mr_oracle_run()
    want, n_want = oracle.rank(traj, capacity=n_traj)
    compare_regions(got, n, want, n_want, w.name)
    # the work counters count what the oracle counts
    assert st["evals"] == ost["evals"] and st["window_evals"] == ost["window_evals"]
    assert st["voxel_visits"] + st["final_visits"] == ost["voxel_visits"]
    top, n2 = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=1000)
    assert n2 == n_want and np.array_equal(top, got[:1000])
    (bg, bn), = ks.ks_detect_batch(ctx, [ks.make_request(t, w.bins, w.spacing, w.scales, w.method, w.max_iter)],
                                   capacity=n_traj)
    assert bn == n and np.array_equal(bg, got)


EDGE_CASES = [
    ("tiny1", np.uint8, (1, 1, 1), 4, 1, (1, 2), 0, 5),
    ("line_x", np.uint16, (1, 1, 37), 8, 3, (1, 4), 1, 10),
    ("flat_z", np.int16, (2, 19, 23), 16, 4, (2, 6), 0, 10),
    ("scale_exceeds_volume", np.uint8, (6, 7, 9), 32, 2, (10, 12), 1, 10),
    ("spacing_exceeds_volume", np.uint8, (9, 10, 11), 32, 50, (1, 3), 0, 10),
    ("max_iter_zero", np.uint8, (20, 21, 22), 32, 5, (2, 4), 1, 0),
    ("bins2", np.uint8, (17, 18, 19), 2, 4, (1, 3), 0, 10),
    ("bins256", np.int16, (17, 18, 33), 256, 5, (2, 5), 1, 10),
    ("bins200_quadrant", np.uint16, (15, 22, 27), 200, 6, (2, 4), 0, 10),
    ("smax32_meanshift", np.uint8, (70, 69, 71), 64, 30, (31, 32), 1, 4),
    ("smax32_quadrant", np.uint8, (70, 69, 67), 64, 40, (31, 32), 0, 3),
    ("smin1_quadrant", np.uint8, (25, 26, 27), 32, 5, (1, 4), 0, 20),
]


@pytest.mark.parametrize("case", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_traces_edge_cases(torch_dev, ctx, case):
    name, dt, shape, bins, sp, scales, method, max_iter = case
    note(f"traces edge {name}")
    hi = 255 if dt == np.uint8 else 4000
    v = random_volume(zlib.crc32(name.encode()) % 1000, shape, dt, 0, hi)
    got = ks.ks_seed_traces(ctx, dev(torch_dev, v), bins, sp, scales, method, max_iter)
    want, _ = oracle.run(v, bins, sp, scales, method, max_iter)
    compare_traces(got, want, name)


def test_constant_volume_finds_nothing(torch_dev, ctx):
    v = np.full((12, 13, 14), 77, np.uint8)
    for method in (ks.KS_QUADRANT, ks.KS_MEANSHIFT):
        note(f"constant volume method={method}")
        regs, n = ks.ks_detect_device(ctx, dev(torch_dev, v), 32, 3, (1, 3), method, 10)
        assert n == 0
        tr = ks.ks_seed_traces(ctx, dev(torch_dev, v), 32, 3, (1, 3), method, 10)
        assert np.all(tr["keep"] == 0)
        assert np.all(tr["iters"] == 0)


# ------------------------------------------------------------------ detect

def compare_regions(got, n_got, want, n_want, label):
    assert n_got == n_want, (label, n_got, n_want)
    assert len(got) == len(want), label
    for f in ("x", "y", "z", "scale", "seed"):
        assert np.array_equal(got[f], want[f]), (label, f)
    assert close32(got["saliency"], want["saliency"]), label
    assert close32(got["entropy"], want["entropy"]), label
    assert close32(got["pdf_change"], want["pdf_change"]), label


@pytest.mark.parametrize("which", ["spheres64", "pet_quadrant", "pet_meanshift"])
def test_detect_matches_oracle(torch_dev, ctx, which):
    w = {"spheres64": synth.spheres_64, "pet_quadrant": lambda: synth.pet_shell(ks.KS_QUADRANT),
         "pet_meanshift": lambda: synth.pet_shell(ks.KS_MEANSHIFT)}[which]()
    note(f"detect {w.name}")
    cap = 100000
    got, n = ks.ks_detect_device(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                 capacity=cap)
    want, n_want, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
    compare_regions(got, n, want, n_want, w.name)
    # truncation: capacity 20 keeps the top 20 and still reports the total
    top, n2 = ks.ks_detect_device(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                  capacity=20)
    assert n2 == n_want and np.array_equal(top, got[:20])


OPTION_CASES = [("rank_w", 0.0, 0.0, 1), ("thresholds", 0.6, 0.02, 0), ("thresholds_rank_w", 1.0, 0.01, 1),
                ("negative_y_min", -1.0, -1.0, 0)]


@pytest.mark.parametrize("method", [ks.KS_QUADRANT, ks.KS_MEANSHIFT])
@pytest.mark.parametrize("case", OPTION_CASES, ids=[c[0] for c in OPTION_CASES])
def test_detect_options_match_oracle(torch_dev, ctx, method, case):
    """Entropy / saliency thresholds and the pdf-change rank key, through the
    context options and through a batch request, against the oracle."""
    name, h_min, y_min, rank_by = case
    w = synth.Workload("opt", synth.spheres_volume(11, (44, 41, 37)), 32, 5, (2, 6), method, 20)
    note(f"detect options {name} method={method}")
    want, n_want, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096,
                                    h_min=h_min, y_min=y_min, rank_by=rank_by)
    opts = ks.options(h_min, y_min, rank_by)
    t = dev(torch_dev, w.volume)
    ks.ks_context_set_options(ctx, opts)
    try:
        got, n = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
    finally:
        ks.ks_context_set_options(ctx, None)
    compare_regions(got, n, want, n_want, name)
    req = ks.make_request(t, w.bins, w.spacing, w.scales, w.method, w.max_iter, opts=opts)
    plain = ks.make_request(t, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    (bg, bn), (pg, pn) = ks.ks_detect_batch(ctx, [req, plain], capacity=4096)
    assert bn == n and np.array_equal(bg, got)
    base, n_base, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=4096)
    compare_regions(pg, pn, base, n_base, "defaults in the same batch")


def test_options_are_validated(torch_dev, ctx):
    for bad in (ks.options(rank_by=2), ks.options(h_min=float("nan")), ks.options(window=(10, 9))):
        with pytest.raises(ks.KsError) as e:
            ks.ks_context_set_options(ctx, bad)
        assert e.value.status == ks.KS_E_INVALID
    bad = ks.options()
    bad.window = 2
    with pytest.raises(ks.KsError):
        ks.ks_context_set_options(ctx, bad)
    # a window level needs bins <= 255 (bin value 255 marks the voxels outside)
    v = dev(torch_dev, random_volume(3, (8, 9, 10), np.uint8, 0, 255))
    ks.ks_context_set_options(ctx, ks.options(window=(10, 200)))
    try:
        with pytest.raises(ks.KsError) as e:
            ks.ks_detect_device(ctx, v, 256, 3, (1, 2), ks.KS_QUADRANT, 5)
        assert e.value.status == ks.KS_E_INVALID
    finally:
        ks.ks_context_set_options(ctx, None)


def test_detect_host_entry_point(torch_dev):
    w = synth.spheres_64()
    note("ks_detect host volume")
    got, n = ks.ks_detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=50)
    want, n_want, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=50)
    compare_regions(got, n, want, n_want, "host")


def test_detect_is_deterministic(torch_dev, ctx):
    w = synth.pet_shell(ks.KS_MEANSHIFT)
    note("determinism")
    t = dev(torch_dev, w.volume)
    a = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=5000)
    b = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=5000)
    assert a[1] == b[1] and np.array_equal(a[0], b[0])


def test_stats_count_the_work(torch_dev, ctx):
    w = synth.spheres_64()
    note("stats")
    ks.ks_detect_device(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    st = ks.ks_last_stats(ctx)
    _, ost = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    assert st["evals"] == ost["evals"]
    assert st["window_evals"] == ost["window_evals"]
    assert st["voxel_visits"] + st["final_visits"] == ost["voxel_visits"]
    assert st["swept_voxels"] == st["voxel_visits"] + st["final_visits"]


def test_stats_meanshift_swept_voxels(torch_dev, ctx):
    """Window evaluations and visits count the method's work (as the oracle does);
    the voxels swept are fewer (first windows shared along a seed's scales, the
    final pass's shell), and fewer again with running-window updates."""
    w = synth.pet_shell(ks.KS_MEANSHIFT)
    note("stats meanshift")
    t = dev(torch_dev, w.volume)
    ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    st = ks.ks_last_stats(ctx)
    ks.ks_context_set_ms_update(ctx, 0)
    try:
        ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter)
        fresh = ks.ks_last_stats(ctx)
    finally:
        ks.ks_context_set_ms_update(ctx, 100)
    for f in ("evals", "window_evals", "voxel_visits", "final_visits", "regions"):
        assert st[f] == fresh[f], f
    assert 0 < fresh["swept_voxels"] < fresh["voxel_visits"] + fresh["final_visits"]
    assert st["swept_voxels"] < 0.7 * fresh["swept_voxels"]


# ---------------------------------------------------------- dense saliency map

MAP_CASES = [
    ("blocks_u8", np.uint8, (17, 21, 26), 16, (2, 4)),
    ("blocks_u16_b64", np.uint16, (13, 19, 23), 64, (1, 3)),
    ("thin_i16", np.int16, (3, 29, 31), 32, (2, 5)),
    ("scale_past_volume", np.uint8, (9, 8, 11), 32, (5, 7)),
    ("b256", np.uint8, (11, 12, 14), 256, (2, 3)),
]


@pytest.mark.parametrize("case", MAP_CASES, ids=[c[0] for c in MAP_CASES])
def test_saliency_map_matches_oracle(torch_dev, ctx, case):
    """Every voxel: s* bit-identical to the oracle's every-voxel search, float32
    saliency within 1e-5 of the accurate value and 0 exactly where it is 0."""
    name, dt, shape, bins, scales = case
    note(f"saliency map {name} {shape} B={bins} s={scales}")
    hi = 255 if dt == np.uint8 else 3000
    v = random_volume(zlib.crc32(name.encode()) % 1000, shape, dt, 0, hi)
    sal, scl = ks.ks_saliency_map(ctx, dev(torch_dev, v), bins, scales)
    torch_dev.cuda.synchronize()
    w_sal, w_scl, _ = oracle.saliency_map(v, bins, scales)
    got_scl = scl.cpu().numpy()
    assert np.array_equal(got_scl, w_scl), int((got_scl != w_scl).sum())
    assert close32(sal.cpu().numpy().ravel(), w_sal.astype(np.float64).ravel())
    assert (w_scl > 0).sum() > 0


def test_saliency_map_spheres64(torch_dev, ctx):
    """The 64^3 spheres volume at its scales 3..8: the whole map against the
    oracle's whole map (about 7 s of CPU)."""
    w = synth.spheres_64()
    note("saliency map spheres64")
    sal, scl = ks.ks_saliency_map(ctx, dev(torch_dev, w.volume), w.bins, w.scales)
    torch_dev.cuda.synchronize()
    got_scl, got_sal = scl.cpu().numpy(), sal.cpu().numpy()
    full_sal, full_scl, _ = oracle.saliency_map(w.volume, w.bins, w.scales)
    assert np.array_equal(got_scl, full_scl), int((got_scl != full_scl).sum())
    assert close32(got_sal.ravel(), full_sal.astype(np.float64).ravel())


# ------------------------------------------------- window level (Sec. 3.2)

WINDOW_CASES = [
    ("u16_pet_window", np.uint16, (21, 26, 31), 32, (1000, 2999)),
    ("i16_narrow", np.int16, (13, 17, 29), 48, (-200, 199)),
    ("u8_empty_corners", np.uint8, (19, 23, 24), 16, (100, 180)),
]


def windowed_volume(name, dt, shape):
    hi = 255 if dt == np.uint8 else 3000
    lo = -900 if dt == np.int16 else 0
    return random_volume(zlib.crc32(name.encode()) % 1000, shape, dt, lo, hi)


@pytest.mark.parametrize("case", WINDOW_CASES, ids=[c[0] for c in WINDOW_CASES])
def test_window_level_binning_and_histograms(torch_dev, ctx, case):
    name, dt, shape, bins, win = case
    note(f"window hooks {name}")
    v = windowed_volume(name, dt, shape)
    bv = oracle.bin_volume(v, bins, window=win)
    pts = positions(v.shape, 12, 5)
    sc = np.random.default_rng(2).integers(1, 9, len(pts)).astype(np.int32)
    ks.ks_context_set_options(ctx, ks.options(window=win))
    try:
        assert np.array_equal(ks.ks_bin_volume(ctx, dev(torch_dev, v), bins), bv)
        cube = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_CUBE, pts, sc)
        ms = ks.ks_histograms(ctx, dev(torch_dev, v), bins, ks.KS_HIST_MEANSHIFT, pts, sc)
    finally:
        ks.ks_context_set_options(ctx, None)
    for i, p in enumerate(pts):
        counts, msum, _, _ = oracle.eval_meanshift(bv, bins, p, int(sc[i]))
        assert np.array_equal(cube[i], counts), (i, p)
        assert np.array_equal(ms[i, 0], counts.astype(np.int32)), (i, p)
        assert np.array_equal(ms[i, 1:].T, msum.astype(np.int32)), (i, p)


@pytest.mark.parametrize("method", [ks.KS_QUADRANT, ks.KS_MEANSHIFT])
@pytest.mark.parametrize("case", WINDOW_CASES, ids=[c[0] for c in WINDOW_CASES])
def test_window_level_traces_and_detection(torch_dev, ctx, case, method):
    """Traces and ranked detections with a window level equal the oracle's."""
    name, dt, shape, bins, win = case
    note(f"window traces {name} method={method}")
    v = windowed_volume(name, dt, shape)
    sp, scales, iters = 4, (2, 5), 20
    t = dev(torch_dev, v)
    ks.ks_context_set_options(ctx, ks.options(window=win))
    try:
        got = ks.ks_seed_traces(ctx, t, bins, sp, scales, method, iters)
        regs, n = ks.ks_detect_device(ctx, t, bins, sp, scales, method, iters, capacity=4096)
    finally:
        ks.ks_context_set_options(ctx, None)
    want, _ = oracle.run(v, bins, sp, scales, method, iters, window=win)
    compare_traces(got, want, f"{name} window")
    wreg, wn, _ = oracle.detect(v, bins, sp, scales, method, iters, capacity=4096, window=win)
    compare_regions(regs, n, wreg, wn, f"{name} window")
    req = ks.make_request(t, bins, sp, scales, method, iters, opts=ks.options(window=win))
    (bg, bn), = ks.ks_detect_batch(ctx, [req], capacity=4096)
    assert bn == n and np.array_equal(bg, regs)


@pytest.mark.parametrize("case", WINDOW_CASES, ids=[c[0] for c in WINDOW_CASES])
def test_window_level_saliency_map(torch_dev, ctx, case):
    name, dt, shape, bins, win = case
    note(f"window map {name}")
    v = windowed_volume(name, dt, shape)
    ks.ks_context_set_options(ctx, ks.options(window=win))
    try:
        sal, scl = ks.ks_saliency_map(ctx, dev(torch_dev, v), bins, (2, 4))
        torch_dev.cuda.synchronize()
    finally:
        ks.ks_context_set_options(ctx, None)
    w_sal, w_scl, _ = oracle.saliency_map(v, bins, (2, 4), window=win)
    assert np.array_equal(scl.cpu().numpy(), w_scl)
    assert close32(sal.cpu().numpy().ravel(), w_sal.astype(np.float64).ravel())


# ------------------------------------------------- explicit seeds (warm start)

def seed_list(shape, n, seed):
    """Random in-volume positions plus the eight corners and a repeated seed."""
    Z, Y, X = shape
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, X, n), rng.integers(0, Y, n), rng.integers(0, Z, n)], 1)
    corners = np.array([(x, y, z) for z in (0, Z - 1) for y in (0, Y - 1) for x in (0, X - 1)])
    return np.concatenate([pts, corners, pts[:1]]).astype(np.int32)


@pytest.mark.parametrize("method", [ks.KS_QUADRANT, ks.KS_MEANSHIFT])
def test_seeded_traces_and_detection_match_oracle(torch_dev, ctx, method):
    w = synth.pet_shell(method)
    seeds = seed_list(w.volume.shape, 150, 71 + method)
    note(f"seeded traces/detect {w.name} n_seeds={len(seeds)}")
    ks.ks_context_set_seeds(ctx, seeds)
    try:
        got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
        regs, n = ks.ks_detect_device(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method,
                                      w.max_iter, capacity=100000)
    finally:
        ks.ks_context_set_seeds(ctx, None)
    want, _ = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, seeds=seeds)
    compare_traces(got, want, f"{w.name} seeded")
    wreg, wn, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, seeds=seeds)
    compare_regions(regs, n, wreg, wn, f"{w.name} seeded")
    # the grid again once the list is cleared
    grid = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
    assert len(grid) == oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)


def test_seeded_edge_cases(torch_dev, ctx):
    v = random_volume(88, (9, 14, 23), np.uint16, 0, 4000)
    Z, Y, X = v.shape
    for method in (ks.KS_QUADRANT, ks.KS_MEANSHIFT):
        note(f"seeded edge cases method={method}")
        try:
            ks.ks_context_set_seeds(ctx, np.zeros((0, 3), np.int32))
            tr = ks.ks_seed_traces(ctx, dev(torch_dev, v), 32, 4, (1, 5), method, 10)
            regs, n = ks.ks_detect_device(ctx, dev(torch_dev, v), 32, 4, (1, 5), method, 10)
            assert len(tr) == 0 and n == 0
            one = np.array([[X - 1, 0, Z // 2]], np.int32)
            ks.ks_context_set_seeds(ctx, one)
            tr = ks.ks_seed_traces(ctx, dev(torch_dev, v), 32, 4, (1, 5), method, 10)
            want, _ = oracle.run(v, 32, 4, (1, 5), method, 10, seeds=one)
            compare_traces(tr, want, f"one seed method={method}")
            for bad in ([X, 0, 0], [0, Y, 0], [0, 0, -1]):
                ks.ks_context_set_seeds(ctx, np.array([bad], np.int32))
                with pytest.raises(ks.KsError):
                    ks.ks_seed_traces(ctx, dev(torch_dev, v), 32, 4, (1, 5), method, 10)
                with pytest.raises(ks.KsError):
                    ks.ks_detect_device(ctx, dev(torch_dev, v), 32, 4, (1, 5), method, 10)
        finally:
            ks.ks_context_set_seeds(ctx, None)
    three = (ctypes.c_int32 * 3)()
    assert ks.lib().ks_context_set_seeds(ctx.handle, three, -1) != 0
    assert ks.lib().ks_context_set_seeds(ctx.handle, None, 5) == 0  # NULL: the grid, count ignored


def test_batch_with_seed_lists(torch_dev, ctx):
    ws = [synth.pet_shell(ks.KS_QUADRANT), synth.pet_shell(ks.KS_MEANSHIFT), synth.spheres_64()]
    vols = [dev(torch_dev, w.volume) for w in ws]
    lists = [seed_list(ws[0].volume.shape, 60, 5), None, np.zeros((0, 3), np.int32), seed_list(ws[1].volume.shape,
                                                                                                 40, 6)]
    order = [0, 1, 2, 1]
    reqs = [ks.make_request(vols[k], ws[k].bins, ws[k].spacing, ws[k].scales, ws[k].method, ws[k].max_iter,
                            seeds=lists[i]) for i, k in enumerate(order)]
    note("batch with seed lists")
    out = ks.ks_detect_batch(ctx, reqs, capacity=100000)
    for i, k in enumerate(order):
        w = ws[k]
        want, wn, _ = oracle.detect(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, seeds=lists[i])
        compare_regions(out[i][0], out[i][1], want, wn, f"batch {i} {w.name}")


# ------------------------------------------------------------------- ABMSOD

def compare_ellipsoids(got, want, label, atol=1e-8):
    """Starts, radii, iterations and stop reasons equal; centres (voxels),
    bandwidths (voxel^2), coefficients and entropies within atol (the GPU takes
    the Gaussian profile along each row by a recurrence anchored on exact exps
    and sums it in 2^-40 fixed point; the oracle takes exp per voxel and sums in
    double)."""
    assert len(got) == len(want), label
    for f in ("x0", "y0", "z0", "radius", "iters", "stop"):
        bad = np.nonzero(got[f] != want[f])[0]
        assert bad.size == 0, f"{label}: {f} differs at {bad[:10]}: got {got[f][bad[:5]]} want {want[f][bad[:5]]}"
    for f in ("x", "h", "rho", "entropy"):
        err = np.abs(np.asarray(got[f], np.float64) - np.asarray(want[f], np.float64))
        assert err.max() <= atol, f"{label}: {f} max error {err.max():.3e}"


def oblique_volume():
    Z, Y, X = 40, 48, 52
    rng = np.random.default_rng(61)
    v = np.clip(np.rint(rng.normal(60, 3, (Z, Y, X))), 0, 255).astype(np.uint8)
    zz, yy, xx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    ax = np.array([1.0, 1.0, 0.5]) / 1.5
    u = np.stack([xx - 26, yy - 24, zz - 20], -1).astype(float)
    along = u @ ax
    perp = np.linalg.norm(u - along[..., None] * ax, axis=-1)
    m = (along / 11) ** 2 + (perp / 3.5) ** 2 <= 1
    v[m] = rng.integers(0, 256, int(m.sum()))
    return v


def test_abmsod_oblique_structure_matches_oracle(torch_dev, ctx):
    v = oblique_volume()
    note("abmsod oblique 52x48x40 spacing 6 radii 3..7")
    ks.ks_context_set_profiling(ctx, True)
    try:
        got = ks.ks_abmsod(ctx, dev(torch_dev, v), 32, 6, (3, 7), 30)
        st = ks.ks_last_stats(ctx)
    finally:
        ks.ks_context_set_profiling(ctx, False)
    want, wst = oracle.abmsod(v, 32, 6, (3, 7), 30)
    compare_ellipsoids(got, want, "oblique")
    assert st["evals"] == wst["evals"] and st["voxel_visits"] == wst["voxel_visits"]
    assert st["trajectories"] == len(want)
    assert np.any(want["stop"] == oracle.ABM_STOP["converged"])


def test_abmsod_window_level_seeds_and_edges(torch_dev, ctx):
    v = random_volume(62, (17, 21, 26), np.uint16, 0, 3000)
    Z, Y, X = v.shape
    seeds = np.array([(0, 0, 0), (X - 1, Y - 1, Z - 1), (13, 10, 8), (2, 19, 15), (13, 10, 8)], np.int32)
    note("abmsod window level, seed list, corners")
    ks.ks_context_set_options(ctx, ks.options(window=(500, 2200)))
    ks.ks_context_set_seeds(ctx, seeds)
    try:
        got = ks.ks_abmsod(ctx, dev(torch_dev, v), 24, 3, (1, 5), 15, threshold=0.002)
        got0 = ks.ks_abmsod(ctx, dev(torch_dev, v), 24, 3, (1, 5), 0)
        ks.ks_context_set_options(ctx, ks.options(window=(3100, 3200)))   # holds no voxel
        empty = ks.ks_abmsod(ctx, dev(torch_dev, v), 24, 3, (1, 5), 15)
    finally:
        ks.ks_context_set_options(ctx, None)
        ks.ks_context_set_seeds(ctx, None)
    want, _ = oracle.abmsod(v, 24, 3, (1, 5), 15, threshold=0.002, seeds=seeds, window=(500, 2200))
    compare_ellipsoids(got, want, "window+seeds")
    want0, _ = oracle.abmsod(v, 24, 3, (1, 5), 0, seeds=seeds, window=(500, 2200))
    compare_ellipsoids(got0, want0, "max_iter 0", atol=0.0)
    assert np.all(empty["stop"] == ks.KS_ABM_EMPTY) and np.all(empty["iters"] == 0)


def test_abmsod_pet_sampled(torch_dev, ctx):
    w = synth.pet_shell(ks.KS_QUADRANT)
    radii, max_iter = (4, 16), 20
    note(f"abmsod {w.name} radii {radii} (full GPU run, sampled oracle)")
    got = ks.ks_abmsod(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, radii, max_iter)
    ids = np.arange(0, len(got), 211)
    want, _ = oracle.abmsod(w.volume, w.bins, w.spacing, radii, max_iter, ids=ids)
    compare_ellipsoids(got[ids], want, w.name)


def test_abmsod_largest_radii_matches_oracle(torch_dev, ctx):
    """Start radii up to 32, the largest allowed: a start window spans 68 slices,
    more than a wavefront's lanes, so a sweep deals its rows in two slice chunks."""
    v = random_volume(64, (72, 40, 44), np.uint8, 0, 255)
    v[20:52, 8:32, 10:34] //= 3          # a darker block: an uneven pmf
    Z, Y, X = v.shape
    seeds = np.array([(22, 20, 36), (5, 30, 60), (40, 2, 10)], np.int32)
    note("abmsod radii 30..32 on 44x40x72, seed list")
    ks.ks_context_set_seeds(ctx, seeds)
    try:
        got = ks.ks_abmsod(ctx, dev(torch_dev, v), 16, 3, (30, 32), 4)
    finally:
        ks.ks_context_set_seeds(ctx, None)
    want, _ = oracle.abmsod(v, 16, 3, (30, 32), 4, seeds=seeds)
    compare_ellipsoids(got, want, "radii 30..32")


def test_abmsod_validation(torch_dev, ctx):
    v = dev(torch_dev, random_volume(63, (8, 9, 10), np.uint8, 0, 255))
    for radii, it, thr in (((0, 3), 5, 0.0), ((4, 3), 5, 0.0), ((1, 33), 5, 0.0), ((1, 3), -1, 0.0),
                           ((1, 3), 5, float("nan"))):
        with pytest.raises(ks.KsError):
            ks.ks_abmsod(ctx, v, 16, 3, radii, it, threshold=thr)


def test_autotune_picks_a_tuning_and_keeps_results(torch_dev, ctx):
    note("autotune on the PET-like volume, both methods")
    try:
        for method in (ks.KS_MEANSHIFT, ks.KS_QUADRANT):
            w = synth.pet_shell(method)
            v = dev(torch_dev, w.volume)
            before = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100000)
            t = ks.ks_context_autotune(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, reps=1)
            assert 3 <= t[0] <= 5 and 2 <= t[1] <= 3 and t[2] in (4, 6, 8) and 0 <= t[3] <= 2, t
            after = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100000)
            assert after[1] == before[1] and np.array_equal(after[0], before[0])
        with pytest.raises(ks.KsError):
            ks.ks_context_autotune(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, reps=0)
    finally:
        restore_tuning(ctx)


def test_plain_c_consumer_matches_oracle(torch_dev, tmp_path):
    """A C99 program linked against libks.so (no Python, no torch) runs ks_detect
    on a host volume; its regions equal the oracle's."""
    import subprocess
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_abi_host import build_consumer
    exe = build_consumer(str(tmp_path))
    for method, scales in ((ks.KS_QUADRANT, (3, 6)), (ks.KS_MEANSHIFT, (2, 5))):
        v = random_volume(91 + method, (26, 30, 34), np.uint16, 0, 3000)
        raw = tmp_path / f"vol{method}.raw"
        v.tofile(raw)
        Z, Y, X = v.shape
        note(f"C consumer method={method}")
        r = subprocess.run([exe, str(raw), "1", str(X), str(Y), str(Z), "32", "5", str(scales[0]), str(scales[1]),
                            str(method), "20", "100000"], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        lines = r.stdout.split("\n")
        n = int(lines[0].split()[1])
        rows = [l.split() for l in lines[1:] if l.strip()]
        want, n_want, _ = oracle.detect(v, 32, 5, scales, method, 20, capacity=100000)
        assert n == n_want and len(rows) == len(want)
        got = np.array([[int(a) for a in row[:5]] for row in rows])
        for k, f in enumerate(("x", "y", "z", "scale", "seed")):
            assert np.array_equal(got[:, k], want[f]), f
        assert close32([float(row[5]) for row in rows], want["saliency"])


@pytest.mark.parametrize("group", [1, 3, 8])
def test_meanshift_scale_groups_give_the_same_traces(torch_dev, ctx, group):
    """A wavefront may run a seed's consecutive scales, each starting from the
    previous first window plus a shell; traces stay bit-identical to the oracle
    (the PET-like volume, and the mean-shift edge cases: clipped windows, windows
    larger than the volume, s up to 32)."""
    ks.ks_context_set_ms_group(ctx, group)
    try:
        w = synth.pet_shell(ks.KS_MEANSHIFT)
        note(f"ms group {group}: {w.name}")
        got = ks.ks_seed_traces(ctx, dev(torch_dev, w.volume), w.bins, w.spacing, w.scales, w.method, w.max_iter)
        ids = np.arange(0, len(got), 3)
        want, _ = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
        compare_traces(got[ids], want, f"{w.name} group {group}")
        for name, dt, shape, bins, sp, scales, method, max_iter in EDGE_CASES:
            if method != ks.KS_MEANSHIFT:
                continue
            note(f"ms group {group}: edge {name}")
            hi = 255 if dt == np.uint8 else 4000
            v = random_volume(zlib.crc32(name.encode()) % 1000, shape, dt, 0, hi)
            got = ks.ks_seed_traces(ctx, dev(torch_dev, v), bins, sp, scales, method, max_iter)
            want, _ = oracle.run(v, bins, sp, scales, method, max_iter)
            compare_traces(got, want, f"{name} group {group}")
        # a window level with groups that cross the replica change at s = 6 -> 7
        v = windowed_volume("group_window", np.uint16, (24, 27, 30))
        note(f"ms group {group}: window level, scales 4..9")
        ks.ks_context_set_options(ctx, ks.options(window=(1000, 2200)))
        try:
            got = ks.ks_seed_traces(ctx, dev(torch_dev, v), 32, 5, (4, 9), ks.KS_MEANSHIFT, 20)
        finally:
            ks.ks_context_set_options(ctx, None)
        want, _ = oracle.run(v, 32, 5, (4, 9), ks.KS_MEANSHIFT, 20, window=(1000, 2200))
        compare_traces(got, want, f"window level group {group}")
    finally:
        ks.ks_context_set_ms_group(ctx, 0)
    with pytest.raises(ks.KsError):
        ks.ks_context_set_ms_group(ctx, 9)


# ------------------------------------------------------ device square roots

def test_device_count_roots_equal_host_for_every_window_count(torch_dev, ctx):
    """The mean-shift decisions take sqrt(c) and 1/sqrt(c) of window counts on the
    device (Sec. 2.3: the bin weights of Eq. 5 and the coefficient).  Both
    operations are correctly rounded in IEEE double, so for every count a window
    can hold (up to the cube of half-width 33, the largest count a table covers)
    they must equal the host's values bit for bit."""
    n = 67 ** 3 + 2
    note(f"device square roots of 0..{n - 1}")
    sq, rs = ks.ks_count_roots(ctx, n)
    c = np.arange(n, dtype=np.float64)
    want_sq = np.sqrt(c)
    with np.errstate(divide="ignore"):
        want_rs = np.where(c > 0, 1.0 / want_sq, 0.0)
    assert np.array_equal(sq.view(np.uint64), want_sq.view(np.uint64))
    assert np.array_equal(rs.view(np.uint64), want_rs.view(np.uint64))
    with pytest.raises(ks.KsError):
        ks.ks_count_roots(ctx, 0)


def test_meanshift_search_in_several_launches(torch_dev, ctx):
    """The mean-shift search split into several launches (each a share of every
    queue's tasks) gives the same traces and detection as one launch, through the
    direct launch sequence and the captured graph."""
    w = synth.pet_shell(ks.KS_MEANSHIFT)
    t = dev(torch_dev, w.volume)
    base_tr = ks.ks_seed_traces(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter)
    base = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100000)
    try:
        for n in (2, 3, 8):
            note(f"mean-shift search in {n} launches")
            ks.ks_context_set_ms_chunks(ctx, n)
            tr = ks.ks_seed_traces(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter)
            assert np.array_equal(tr, base_tr), n
            got = ks.ks_detect_device(ctx, t, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100000)
            assert got[1] == base[1] and np.array_equal(got[0], base[0]), n
            (bg, bn), = ks.ks_detect_batch(ctx, [ks.make_request(t, w.bins, w.spacing, w.scales, w.method,
                                                                 w.max_iter)], capacity=100000)
            assert bn == base[1] and np.array_equal(bg, base[0]), n
        for bad in (0, 9):
            with pytest.raises(ks.KsError):
                ks.ks_context_set_ms_chunks(ctx, bad)
    finally:
        ks.ks_context_set_ms_chunks(ctx, 1)
