"""The oracle's run of every trajectory of the MR-like workload (256x256x160
int16, 64 bins, spacing 8, scales 4..24, mean-shift, 100 iterations: 430,080
trajectories, several minutes on one core), sharded by trajectory id over host
processes.

The pool is forked when collection ends, before any test has touched the GPU
(a process must not fork once HIP is initialised), and works while the other
tests run; the full-size parity tests wait for its result.  Test
infrastructure only: nothing here runs a kernel.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

# tests that need the full oracle run
USERS = ("test_traces_mr_blobs_full", "test_detect_mr_blobs_full_matches_oracle")
JOBS = 96   # shards; more than workers, so that uneven shards balance

_pool = None
_async = None
_t0 = 0.0


def _shard(job):
    import oracle
    from paper_1310_6736_amd import synth

    k, jobs = job
    w = synth.mr_blobs()
    n = oracle.num_trajectories(w.dims, w.spacing, w.scales, w.method)
    ids = np.arange(k, n, jobs, dtype=np.int64)
    arr, st = oracle.run(w.volume, w.bins, w.spacing, w.scales, w.method, w.max_iter, ids=ids)
    return ids, arr, st


def workers() -> int:
    # the GPU machine gives a process 16 host cores whatever the machine reports
    return max(1, min(16, os.cpu_count() or 1))


def start():
    """Forks the pool and queues every shard (no-op if already started)."""
    global _pool, _async, _t0
    if _pool is not None:
        return
    _t0 = time.perf_counter()
    _pool = mp.get_context("fork").Pool(workers())
    _async = _pool.map_async(_shard, [(k, JOBS) for k in range(JOBS)], chunksize=1)
    _pool.close()


def started() -> bool:
    return _pool is not None


_result = None


def result(timeout=1800.0):
    """(trajectory records of the whole run in trajectory-id order, stats dict,
    wall seconds the pool took)."""
    global _result
    if _result is None:
        if _async is None:
            raise RuntimeError("the oracle pool was not started at collection")
        parts = _async.get(timeout)
        wall = time.perf_counter() - _t0
        ids = np.concatenate([p[0] for p in parts])
        arr = np.concatenate([p[1] for p in parts])
        order = np.argsort(ids, kind="stable")
        assert np.array_equal(ids[order], np.arange(ids.size))
        st = {f: sum(p[2][f] for p in parts) for f in parts[0][2]}
        _result = (arr[order], st, wall)
        _pool.join()
    return _result


def stop():
    global _pool
    if _pool is not None:
        _pool.terminate()
        _pool.join()
        _pool = None
