"""Batched form (sdbg_batch_run) against the oracle and the single-set path.

Every set's edges and SdBG arrays must equal the oracle's for that set
alone, bit for bit, whatever the grouping of sets into passes (memory
budget), the mix of host and device inputs, or the key width."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import assert_graph_equal, say, to_device
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu


def _sets(seed: int, n: int, k: int):
    """Uneven sets: empty, shorter than k+1, single read, 'N' bytes, and
    sets spanning several extraction tiles."""
    out = []
    rng = np.random.default_rng(seed)
    for i in range(n):
        kind = i % 7
        if kind == 0:
            rs = synth.from_strings([], k)
        elif kind == 1:
            rs = synth.from_strings(["ACGT" * ((k // 4) or 1)], k)  # fewer than k+1 bases when k % 4 == 3
        elif kind == 2:
            rs = synth.random_small(1, k + 1, k + 30, 200, 0.0, seed * 100 + i)
        else:
            nr = int(rng.integers(5, 60 if kind < 5 else 400))
            rs = synth.random_small(nr, k + 1, k + 90, int(rng.integers(300, 3000)), 0.01, seed * 100 + i,
                                    n_rate=0.002 if kind == 6 else 0.0)
        out.append(rs)
    return out


def _check_against_oracle(sets, results, k, d, mercy):
    for i, (rs, (e, g)) in enumerate(zip(sets, results)):
        o = oracle.count_solid(rs.seq, rs.offsets, k, d, mercy)
        keys, cnt = e.to_host()
        assert e.n_occ == o.n_occ, i
        assert np.array_equal(keys, o.keys), i
        assert np.array_equal(cnt, o.counts), i
        assert e.n_mercy == o.n_mercy, i
        if g is not None:
            assert_graph_equal(g.to_host(), oracle.build_graph(o.keys, o.counts, k))


def _close(results):
    for e, g in results:
        e.close()
        if g is not None:
            g.close()


@pytest.mark.parametrize("k", [21, 31, 41, 63, 81, 99])
def test_batch_matches_oracle(k):
    say(f"batch k={k}")
    sets = _sets(k, 23, k)
    dev = [to_device(rs) for rs in sets]
    res = sdbg.batch_run(dev, k, 2, False)
    _check_against_oracle(sets, res, k, 2, False)
    _close(res)


@pytest.mark.parametrize("d", [1, 3])
def test_batch_thresholds(d):
    say(f"batch d={d}")
    sets = _sets(500 + d, 15, 31)
    res = sdbg.batch_run([to_device(rs) for rs in sets], 31, d, False)
    _check_against_oracle(sets, res, 31, d, False)
    _close(res)


def test_batch_waves_and_host_inputs():
    """A small budget splits the sets into several passes; host and device
    inputs mixed; results identical to one pass."""
    k = 31
    sets = _sets(77, 30, k)
    mixed = [(rs.seq, rs.offsets) if i % 2 else to_device(rs) for i, rs in enumerate(sets)]
    one = sdbg.batch_run(mixed, k, 2, False)
    occ = [rs.n_windows(k) * 2 for rs in sets]
    budget = max(occ) * 48 + 4096  # about one set per pass
    say(f"batch waves budget={budget}")
    many = sdbg.batch_run(mixed, k, 2, False, mem_budget=budget)
    for (e1, g1), (e2, g2) in zip(one, many):
        k1, c1 = e1.to_host()
        k2, c2 = e2.to_host()
        assert np.array_equal(k1, k2) and np.array_equal(c1, c2)
        assert_graph_equal(g1.to_host(), g2.to_host())
    _check_against_oracle(sets, many, k, 2, False)
    _close(one)
    _close(many)


def test_batch_mercy_uses_single_set_path():
    k = 21
    sets = [synth.random_small(40, 30, 90, 400, 0.02, 900 + i) for i in range(6)]
    res = sdbg.batch_run([to_device(rs) for rs in sets], k, 2, True)
    _check_against_oracle(sets, res, k, 2, True)
    _close(res)


def test_batch_equals_single_calls_on_workload_sets():
    """Sets of the 4096-set workload recipe (read counts scaled down)."""
    sets = [synth.batch_set(i, read_scale=0.01) for i in range(12)]
    say("batch workload sets: " + ", ".join(str(rs.n_reads) for rs in sets))
    res = sdbg.batch_run([to_device(rs) for rs in sets], 31, 2, False)
    for rs, (e, g) in zip(sets, res):
        seq, off = to_device(rs)
        e1 = sdbg.count_solid(seq, off, 31, 2, False)
        g1 = sdbg.build(e1)
        k1, c1 = e1.to_host()
        k2, c2 = e.to_host()
        assert e1.n_occ == e.n_occ
        assert np.array_equal(k1, k2) and np.array_equal(c1, c2)
        assert_graph_equal(g.to_host(), g1.to_host())
        e1.close()
        g1.close()
    _check_against_oracle(sets[:4], res[:4], 31, 2, False)
    _close(res)


def test_batch_edges_only_and_empty():
    assert sdbg.batch_run([], 31) == []
    sets = [synth.from_strings([], 31), synth.from_strings(["ACGT"], 31)]
    res = sdbg.batch_run([to_device(rs) for rs in sets], 31, 2, False, build=False)
    for e, g in res:
        assert g is None and e.n == 0 and e.n_occ == 0
        e.close()


TUNES = [
    {"digit_bits": 4, "tile_shift": 1, "leaf_wg_per_cu": 1, "leaf_cap_shift": 1, "first_bits": 4},
    {"digit_bits": 6, "tile_shift": 0, "leaf_wg_per_cu": 4, "leaf_cap_shift": 0, "first_bits": 7},
    {"digit_bits": 7, "tile_shift": 1, "leaf_wg_per_cu": 32, "leaf_cap_shift": 1, "first_bits": 8},
]


@pytest.mark.parametrize("k", [31, 41, 99])
def test_launch_parameters_do_not_change_results(k):
    """Every autotuner candidate gives the same bytes (batched and plain)."""
    sets = _sets(300 + k, 12, k)
    big = synth.metagenome_long(scale=0.001, k=k)
    dev = [to_device(rs) for rs in sets]
    bseq, boff = to_device(big)
    sdbg.tune_set(None)
    ref = sdbg.batch_run(dev, k, 2, False)
    ref_keys = [e.to_host() for e, _ in ref]
    e0 = sdbg.count_solid(bseq, boff, k, 2, True)
    big_ref = e0.to_host()
    try:
        for t in TUNES:
            say(f"tune {t} k={k}")
            sdbg.tune_set(t)
            assert all(sdbg.tune_get()[key] == val for key, val in t.items())
            res = sdbg.batch_run(dev, k, 2, False)
            for (e, g), (rk, rc), (_, rg) in zip(res, ref_keys, ref):
                kk, cc = e.to_host()
                assert np.array_equal(kk, rk) and np.array_equal(cc, rc)
                assert_graph_equal(g.to_host(), rg.to_host())
            _close(res)
            e1 = sdbg.count_solid(bseq, boff, k, 2, True)
            kk, cc = e1.to_host()
            assert np.array_equal(kk, big_ref[0]) and np.array_equal(cc, big_ref[1])
            e1.close()
    finally:
        sdbg.tune_set(None)
    e0.close()
    _close(ref)


def test_autotune_keeps_results():
    sets = [synth.batch_set(i, read_scale=0.003) for i in range(64)]
    dev = [to_device(rs) for rs in sets]
    sdbg.tune_set(None)
    ref = sdbg.batch_run(dev, 31, 2, False, build=False)
    try:
        best = sdbg.autotune(dev, 31, reps=1)
        say(f"autotune picked {best}")
        assert best == sdbg.tune_get()
        assert best["digit_bits"] in (6, 7, 8) and best["tile_shift"] in (0, 1)
        assert best["leaf_wg_per_cu"] in (4, 8, 16, 32) and best["leaf_cap_shift"] in (0, 1)
        res = sdbg.batch_run(dev, 31, 2, False, build=False)
        for (e, _), (r, _) in zip(res, ref):
            a, b = e.to_host(), r.to_host()
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        _close(res)
    finally:
        sdbg.tune_set(None)
    _close(ref)


def test_autotune_writes_only_its_struct():
    """sdbg_autotune fills every field of the caller's sdbg_tune (including
    mercy_shift) and writes nothing past its end."""
    import ctypes

    lib = sdbg.load()
    sdbg._tune_api(lib)
    sets = [synth.batch_set(i, read_scale=0.002) for i in range(8)]
    dev = [to_device(rs) for rs in sets]
    arr = (sdbg._Reads * len(dev))()
    keep = []
    for i, (seq, off) in enumerate(dev):
        r, kp = sdbg._reads_struct(seq, off)
        arr[i] = r
        keep += kp
    size = ctypes.sizeof(sdbg._Tune)
    raw = (ctypes.c_uint8 * (size + 64))(*([0xAB] * (size + 64)))
    p = sdbg._Params(31, 2, 0, 8, 0, None)
    try:
        sdbg.tune_set({"mercy_shift": 3})
        rc = lib.sdbg_autotune(arr, len(dev), ctypes.byref(p), 1, ctypes.cast(raw, ctypes.POINTER(sdbg._Tune)))
        assert rc == 0, lib.sdbg_last_error()
        assert bytes(raw[size:]) == b"\xab" * 64
        t = ctypes.cast(raw, ctypes.POINTER(sdbg._Tune)).contents
        assert sdbg._tune_dict(t) == sdbg.tune_get()
        assert t.mercy_shift == 3 and list(t.reserved) == [0, 0]
    finally:
        sdbg.tune_set(None)


def test_batch_rejects_bad_device_offsets():
    """Offsets of device-resident sets are checked on the device: a first
    offset other than 0, or offsets that decrease, give SDBG_E_INVAL and no
    outputs."""
    import torch

    good = synth.random_small(20, 30, 60, 300, 0.0, 5)
    seq, off = to_device(good)
    for case in ("first", "decreasing"):
        o = off.clone()
        if case == "first":
            o[0] = 5
        else:
            o[3] = o[4] + 7  # offsets[3] > offsets[4]
        with pytest.raises(sdbg.SdbgError):
            sdbg.batch_run([(seq, off), (seq, o)], 21, 2, False)
    torch.cuda.synchronize()
    res = sdbg.batch_run([(seq, off)], 21, 2, False)
    _check_against_oracle([good], res, 21, 2, False)
    _close(res)
