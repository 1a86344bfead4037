"""Host-only tests of the request loop's admission policy
(paper_1409_7208_amd/csrc/admission.h) against a mock executor
(tests/sched_mock.cpp), built with AddressSanitizer and
UndefinedBehaviorSanitizer.  No GPU is involved: jobs "run" on a fake device
of fixed memory, so admission, the out-of-memory re-queue to run alone,
FIFO order and termination are checked on arrival traces shaped like the
serving workload."""

from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1409_7208_amd import sdbg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
GB = 10**9


@pytest.fixture(scope="module")
def mock_bin(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("sched") / "sched_mock")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_1409_7208_amd", "csrc"), os.path.join(HERE, "sched_mock.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def run_mock(binary, budget, device, workers, jobs, scale, exclusive_above=0):
    lines = [f"{budget} {device} {workers} {scale} {exclusive_above}"]
    lines += [f"{a:.6f} {fp} {peak} {dur:.6f}" for a, fp, peak, dur in jobs]
    r = subprocess.run([binary], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, f"mock exit {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    rows = [list(map(int, ln.split())) for ln in r.stdout.splitlines() if ln and ln != "ok"]
    assert r.stdout.rstrip().endswith("ok")
    return rows  # id, status, attempts, first_start_rank


def serving_trace_footprints(rates=(1.0, 2.0, 5.0), pool=32, read_scale=0.5, genome_scale=0.1):
    """Arrivals and footprints of the serving benchmark's replays up to the
    given rates (pool jobs reused round robin), footprints from the
    library's own admission formula."""
    shapes = synth.serving_job_shapes(pool, read_scale=read_scale, genome_scale=genome_scale)
    fps = []
    for n, L, k in shapes:
        off = np.arange(n + 1, dtype=np.uint64) * np.uint64(L)
        fps.append(sdbg.job_footprint(np.zeros(1, dtype=np.uint8), off, k))
    occ = [2 * n * max(0, L - k) for n, L, k in shapes]
    rng = np.random.default_rng(0x14097208)
    traces = []
    for lam in rates:
        n = int(min(pool, max(8, 4 * lam)))
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n))
        arr -= arr[0]
        traces.append([(float(arr[i]), fps[i % pool], occ[i % pool]) for i in range(n)])
    return traces


@pytest.mark.parametrize("peak_factor", [0.5, 1.0, 2.0, 4.0])
def test_serving_trace_replay_terminates(mock_bin, peak_factor):
    """The replays up to 5 jobs/s, 4 workers, a 288 GB device with an 80%
    budget; true peaks a multiple of the footprint (above 1: the
    footprint undercounts and jobs run out of memory next to others)."""
    device = 288 * GB
    budget = int(0.8 * device)
    for trace in serving_trace_footprints():
        jobs = [(a, fp, int(fp * peak_factor), occ / 20e9) for a, fp, occ in trace]
        rows = run_mock(mock_bin, budget, device, 4, jobs, scale=0.05, exclusive_above=8 << 30)
        for (a, fp, peak, _), (_, status, attempts, _) in zip(jobs, rows):
            if peak <= device:
                assert status == 0, (fp, peak, status)
            else:
                assert status == -3
            assert 1 <= attempts <= 2


def test_random_traces(mock_bin):
    rng = np.random.default_rng(7)
    for rep in range(6):
        n = 200
        device = 100 * GB
        budget = int(device * rng.uniform(0.5, 1.0))
        fp = (np.exp(rng.uniform(np.log(0.1), np.log(1.5), n)) * budget).astype(np.int64)
        peak = (fp * rng.uniform(0.2, 3.0, n)).astype(np.int64)
        arr = np.cumsum(rng.exponential(0.002, n))
        dur = rng.uniform(0.0005, 0.01, n)
        workers = int(rng.integers(1, 9))
        excl = int(budget * rng.uniform(0.2, 0.6)) if rep % 2 else 0  # large jobs run alone
        rows = run_mock(mock_bin, budget, device, workers, list(zip(arr, fp, peak, dur)), scale=1.0,
                        exclusive_above=excl)
        for (i, status, attempts, first), p in zip(rows, peak):
            assert status == (0 if p <= device else -3)
            assert attempts in (1, 2)
        firsts = [r[3] for r in rows]
        assert firsts == sorted(firsts)  # first attempts in submission order


def test_footprint_call_is_host_only():
    off = np.array([0, 100, 250], dtype=np.uint64)
    b21 = sdbg.job_footprint(np.zeros(250, dtype=np.uint8), off, 21)
    b61 = sdbg.job_footprint(np.zeros(250, dtype=np.uint8), off, 61)
    assert b61 > b21 > 0
    with pytest.raises(sdbg.SdbgError):
        sdbg.job_footprint(np.zeros(250, dtype=np.uint8), off, 1)
