"""Served form (sdbg_server_*): each job's result is the same alone and in
the mix, bit for bit, and the request loop's admission, queue and cancel
rules hold."""

from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from gpu_util import assert_graph_equal, say, to_device
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu


def _jobs(n: int, seed: int):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        k = int(rng.choice([21, 41, 61]))
        nr = int(rng.integers(50, 3000))
        rs = synth.random_small(nr, 100, 150, int(rng.integers(2000, 40000)), 0.005, seed * 1000 + j)
        out.append((rs, k))
    return out


def _alone(rs, k):
    seq, off = to_device(rs)
    e = sdbg.count_solid(seq, off, k, 2, True)
    g = sdbg.build(e)
    keys, cnt = e.to_host()
    h = g.to_host()
    res = (e.n_occ, e.n_mercy, keys, cnt, h)
    e.close()
    g.close()
    return res


def _same(res: sdbg.JobResult, ref):
    n_occ, n_mercy, keys, cnt, h = ref
    assert res.status == 0, res.error
    k2, c2 = res.edges.to_host()
    assert res.edges.n_occ == n_occ and res.edges.n_mercy == n_mercy and res.n_occ == n_occ
    assert np.array_equal(k2, keys) and np.array_equal(c2, cnt)
    assert_graph_equal(res.graph.to_host(), h)


@pytest.mark.parametrize("max_jobs", [1, 4])
def test_server_results_equal_alone(max_jobs):
    jobs = _jobs(12, 7 + max_jobs)
    refs = [_alone(rs, k) for rs, k in jobs]
    say(f"server max_jobs={max_jobs}: {len(jobs)} jobs submitted at once")
    with sdbg.Server(max_jobs=max_jobs) as srv:
        ids = [srv.submit(rs.seq, rs.offsets, k, 2, True) for rs, k in jobs]
        results = [srv.poll(i) for i in ids]
    for res, ref in zip(results, refs):
        _same(res, ref)
        assert res.submit_s <= res.start_s <= res.end_s
        res.edges.close()
        res.graph.close()
    # one job checked against the oracle as well
    rs, k = jobs[0]
    o = oracle.count_solid(rs.seq, rs.offsets, k, 2, True)
    assert np.array_equal(refs[0][2], o.keys) and np.array_equal(refs[0][3], o.counts)


def test_server_overlaps_jobs_and_respects_budget():
    """With room for two jobs, two run at once; with a budget below one
    job's footprint, jobs run one at a time (each alone)."""
    jobs = _jobs(6, 99)
    with sdbg.Server(max_jobs=4) as srv:
        ids = [srv.submit(rs.seq, rs.offsets, k, 2, True) for rs, k in jobs]
        res = [srv.poll(i) for i in ids]
    spans = [(r.start_s, r.end_s) for r in res]
    assert all(r.status == 0 for r in res)
    with sdbg.Server(max_jobs=4, mem_budget=1 << 20) as srv:
        ids = [srv.submit(rs.seq, rs.offsets, k, 2, True) for rs, k in jobs]
        res2 = [srv.poll(i) for i in ids]
    assert all(r.status == 0 for r in res2)
    spans2 = sorted((r.start_s, r.end_s) for r in res2)
    for (a0, a1), (b0, b1) in zip(spans2, spans2[1:]):
        assert b0 >= a1  # never two at once
    for r1, r2 in zip(res, res2):
        k1, c1 = r1.edges.to_host()
        k2, c2 = r2.edges.to_host()
        assert np.array_equal(k1, k2) and np.array_equal(c1, c2)
        assert_graph_equal(r1.graph.to_host(), r2.graph.to_host())
    say(f"spans shared budget: {spans}")


def test_server_queue_full_cancel_and_stop():
    big = synth.metagenome(scale=0.1)  # 1M reads: runs long enough to hold the one worker
    small = synth.random_small(100, 100, 120, 5000, 0.005, 5)
    with sdbg.Server(max_jobs=1, queue_cap=1) as srv:
        j1 = srv.submit(big.seq, big.offsets, 31, 2, True)
        t0 = time.time()
        while srv.poll(j1, wait=False).status == 1 and time.time() - t0 < 30:
            time.sleep(0.001)  # waiting -> running (a finished job would be handed over here)
        j2 = srv.submit(small.seq, small.offsets, 21)
        with pytest.raises(sdbg.SdbgError) as ei:
            srv.submit(small.seq, small.offsets, 21)
        assert ei.value.code == -5
        assert srv.cancel(j2) == 0
        r2 = srv.poll(j2)
        assert r2.status == -6 and r2.edges is None
        r1 = srv.poll(j1, wait=False)
        if r1.status == 2:
            assert srv.cancel(j1) == -5
            r1 = srv.poll(j1)
        assert r1.status == 0
        r1.edges.close()
        r1.graph.close()
        with pytest.raises(sdbg.SdbgError):
            srv.poll(j1)  # forgotten after it was handed over
        # results left unpolled are freed by stop
        srv.submit(small.seq, small.offsets, 21)


def test_server_bad_input():
    with sdbg.Server(max_jobs=2) as srv:
        rs = synth.random_small(10, 50, 60, 500, 0.0, 3)
        with pytest.raises(sdbg.SdbgError) as ei:
            srv.submit(rs.seq, rs.offsets, 200)
        assert ei.value.code == -1
        seq, off = to_device(rs)
        with pytest.raises(sdbg.SdbgError):
            srv.submit(seq, off, 21)  # device reads are not taken
        e = srv.submit(synth.from_strings([], 21).seq, synth.from_strings([], 21).offsets, 21)
        r = srv.poll(e)
        assert r.status == 0 and r.edges.n == 0 and r.graph.m == 0


@pytest.mark.parametrize("k", [21, 41, 61, 81, 99])
def test_footprint_covers_peak_device_memory(k):
    """The footprint a job is admitted with bounds the library's device
    memory at the job's peak (pool bytes in use, outputs included)."""
    cases = [synth.metagenome(scale=0.01), synth.tiny(scale=0.5),
             synth.random_small(3000, 100, 150, 3000, 0.005, 11), synth.metagenome_long(scale=0.01)]
    with sdbg.Server(max_jobs=1) as srv:
        for rs in cases:
            base = sdbg.pool_stats(reset_peak=True)["in_use"]
            r = srv.poll(srv.submit(rs.seq, rs.offsets, k, 2, True))
            assert r.status == 0, r.error
            peak = sdbg.pool_stats()["peak"] - base
            say(f"k={k} {rs.n_reads} reads: peak {peak} bytes, footprint {r.footprint} ({peak / r.footprint:.2f})")
            r.edges.close()
            r.graph.close()
            assert peak <= r.footprint


def test_injected_allocation_failures_leave_no_trace():
    """A device allocation that fails at any point of a call returns
    SDBG_E_NOMEM_DEVICE, releases everything the call held, and the next
    call's result is unchanged; in the request loop the job fails alone."""
    rs = synth.tiny(scale=0.05)
    ref = _alone(rs, 21)
    seq, off = to_device(rs)
    import torch

    torch.cuda.synchronize()
    base = sdbg.pool_stats()["in_use"]
    failed = 0
    try:
        for after in [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]:
            sdbg.fail_alloc_after(after)
            say(f"allocation {after + 1} fails")
            e = None
            try:
                e = sdbg.count_solid(seq, off, 21, 2, True)
                sdbg.build(e).close()
            except sdbg.SdbgError as err:
                assert err.code == -3 and "injected" in str(err)
                failed += 1
            finally:
                if e is not None:
                    e.close()
            sdbg.fail_alloc_after(-1)
            assert sdbg.pool_stats()["in_use"] == base
    finally:
        sdbg.fail_alloc_after(-1)
    assert failed >= 5
    res = _alone(rs, 21)
    assert res[0] == ref[0] and res[1] == ref[1]
    assert np.array_equal(res[2], ref[2]) and np.array_equal(res[3], ref[3])
    assert_graph_equal(res[4], ref[4])
    with sdbg.Server(max_jobs=2) as srv:
        sdbg.fail_alloc_after(4)
        try:
            bad = srv.poll(srv.submit(rs.seq, rs.offsets, 21, 2, True))
        finally:
            sdbg.fail_alloc_after(-1)
        assert bad.status == -3
        good = srv.poll(srv.submit(rs.seq, rs.offsets, 21, 2, True))
        _same(good, ref)
        good.edges.close()
        good.graph.close()
