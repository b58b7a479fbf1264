"""The allocation-free detection entry point against ks_detect_device, through
the C ABI: same regions bit for bit and the same work counters, call after call
on the one static device array (the later calls on smaller inputs than the
first, so stale contents of a larger call would show), and the size limit."""
import sys

import numpy as np
import pytest

from paper_1310_6736_amd import ks, synth

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_equals_detect_device_call_after_call(torch_dev):
    ctx = ks.Context(0)
    try:
        cases = [(synth.mr_blobs(), 2048), (synth.pet_shell(ks.KS_MEANSHIFT), 100000),
                 (synth.spheres_64(), 4096), (synth.pet_shell(ks.KS_QUADRANT), 300), (synth.mr_blobs(), 64)]
        for w, cap in cases:
            note(f"noalloc {w.name} capacity {cap}")
            v = torch_dev.from_numpy(w.volume).to("cuda:0")
            got = ks.ks_detect_device_noalloc(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                              capacity=cap)
            st_got = ks.ks_last_stats(ctx)
            want = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=cap)
            st_want = ks.ks_last_stats(ctx)
            assert got[1] == want[1] and np.array_equal(got[0], want[0]), w.name
            for f in ("trajectories", "evals", "window_evals", "voxel_visits", "final_visits", "regions",
                      "swept_voxels", "lds_ops"):
                assert st_got[f] == st_want[f], (w.name, f)
    finally:
        ctx.close()


def test_noalloc_rejects_work_beyond_the_array(torch_dev):
    ctx = ks.Context(0)
    try:
        w = synth.spheres_64()
        v = torch_dev.from_numpy(w.volume).to("cuda:0")
        note("noalloc beyond the array")
        with pytest.raises(ks.KsError) as e:
            # 3.3 million region slots (105.6 MB of results) do not fit 96 MiB
            ks.ks_detect_device_noalloc(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter,
                                        capacity=3_300_000)
        assert e.value.status == ks.KS_E_TOO_LARGE
        # and the array still serves the next call
        got = ks.ks_detect_device_noalloc(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100)
        want = ks.ks_detect_device(ctx, v, w.bins, w.spacing, w.scales, w.method, w.max_iter, capacity=100)
        assert got[1] == want[1] and np.array_equal(got[0], want[0])
    finally:
        ctx.close()
