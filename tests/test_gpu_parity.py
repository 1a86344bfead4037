"""Parity of the HIP path (through the C ABI) with the CPU oracle.

All results are integers, so the bar is bit-exact equality: edge keys,
counts, mercy count, occurrence count and every SdBG array."""

from __future__ import annotations

import json
import os

import numpy as np
import pytest

import brute
import oracle
from gpu_util import assert_graph_equal, gpu_count, gpu_graph, graph_invariants, revcomp_keys_w1, say
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "toys.json")) as f:
    TOYS = json.load(f)["toys"]


def _bits_to_int(words) -> int:
    return sum(int(w) << (64 * i) for i, w in enumerate(words))


def _parity(rs, k, d, mercy, **kw):
    say(f"case {rs.name} k={k} d={d} mercy={mercy} {kw}")
    e, keys, cnt = gpu_count(rs, k, d, mercy, **kw)
    o = oracle.count_solid(rs.seq, rs.offsets, k, d, mercy)
    assert e.n_occ == o.n_occ
    assert keys.shape == o.keys.shape
    assert np.array_equal(keys, o.keys)
    assert np.array_equal(cnt, o.counts)
    assert e.n_mercy == o.n_mercy
    h = gpu_graph(e)
    og = oracle.build_graph(o.keys, o.counts, k)
    assert_graph_equal(h, og)
    e.close()
    graph_invariants(h, o.keys.shape[0])
    return h


@pytest.mark.parametrize("toy", TOYS, ids=[t["name"] for t in TOYS])
def test_toys(toy):
    rs = synth.from_strings(toy["reads"], toy["k"], toy["d"], toy["mercy"])
    e, keys, cnt = gpu_count(rs, toy["k"], toy["d"], toy["mercy"])
    assert keys[:, -1].tolist() == toy["keys"]
    assert cnt.tolist() == toy["counts"]
    assert e.n_mercy == toy["n_mercy"] and e.n_occ == toy["n_occ"]
    h = gpu_graph(e)
    assert h.m == toy["m"] and h.t == toy["t"]
    assert h.W.tolist() == toy["W"]
    assert _bits_to_int(h.last) == int(toy["last"], 16)
    assert _bits_to_int(h.valid) == int(toy["valid"], 16)
    assert _bits_to_int(h.tip) == int(toy["tip"], 16)
    assert h.mult.tolist() == toy["mult"]
    assert h.F.tolist() == toy["F"]
    assert _bits_to_int(h.tip_seq) == int(toy["tip_seq"], 16)


def _random_cases():
    cases = []
    for seed in range(16):
        k = [2, 3, 5, 7, 11, 15][seed % 6]
        d = [1, 2, 3][seed % 3]
        cases.append((seed, k, d, seed % 2 == 0, 0.05 if seed % 4 == 1 else 0.0))
    cases += [(100, 31, 2, True, 0.0), (101, 32, 2, True, 0.02), (102, 47, 3, True, 0.0), (103, 63, 2, False, 0.0),
              (104, 64, 2, True, 0.01), (105, 81, 2, True, 0.0), (106, 95, 1, False, 0.0), (107, 96, 2, True, 0.0),
              (108, 99, 2, True, 0.01), (109, 127, 2, True, 0.0)]
    return cases


@pytest.mark.parametrize("seed,k,d,mercy,n_rate", _random_cases())
def test_random_small(seed, k, d, mercy, n_rate):
    glen = 60 if k < 8 else 4 * k
    rs = synth.random_small(60, k, k + 40, glen, 0.03, seed, n_rate=n_rate)
    rs.name = f"random_small({seed})"
    h = _parity(rs, k, d, mercy)
    nodes, edges = brute.decode_sdbg(h.W, h.last, h.valid, h.tip, h.mult, h.F, h.tip_seq, h.m, k)
    E, _ = brute.brute_edges(rs.reads(), k, d, mercy)
    assert edges == E


@pytest.mark.parametrize("mercy", [False, True])
def test_tiny_workload(mercy):
    """50 kb genome, 20,000 reads of 100 bp, 1% errors, k=21, d=2."""
    _parity(synth.tiny(), 21, 2, mercy)


@pytest.mark.parametrize("k", [21, 31, 33, 41, 61, 64, 75, 81, 95, 96, 99, 127])
def test_metagenome_shape_each_k(k):
    """Skewed community (log-normal abundance), scaled down so the oracle
    finishes quickly; every key width (1-4 words) at the ends of its k
    range.  Thousands of workgroups per launch, so a kernel that is only
    right in the first wave of workgroups on each CU fails here."""
    rs = synth.metagenome_long(scale=0.0015, k=k)
    _parity(rs, k, 2, True)


def test_host_and_device_inputs_agree():
    rs = synth.random_small(200, 30, 80, 400, 0.02, 5, n_rate=0.01)
    _, k1, c1 = gpu_count(rs, 13, 2, True, device_input=True)
    _, k2, c2 = gpu_count(rs, 13, 2, True, device_input=False)
    assert np.array_equal(k1, k2) and np.array_equal(c1, c2)


@pytest.mark.parametrize("k", [21, 33])
def test_independent_of_prefix_len_and_budget(k):
    """Block-wise grouping (Section 2, second paragraph) must not change
    the result: small budgets force many groups of prefix blocks."""
    rs = synth.tiny(scale=0.5)
    ref_e, ref_k, ref_c = gpu_count(rs, k, 2, True)
    ref_h = gpu_graph(ref_e)
    n_occ = ref_e.n_occ
    w = sdbg.key_words(k)
    for pl, frac in [(0, 0), (4, 3), (8, 7), (8, 23), (6, 11)]:
        budget = 0 if frac == 0 else int(n_occ * (16 * w + 4) / frac) + 1
        say(f"prefix_len={pl} budget={budget}")
        e, kk, cc = gpu_count(rs, k, 2, True, prefix_len=pl, mem_budget=budget)
        assert np.array_equal(kk, ref_k) and np.array_equal(cc, ref_c)
        assert_graph_equal(gpu_graph(e), ref_h)


def test_budget_too_small_is_an_error():
    rs = synth.tiny(scale=0.05)
    with pytest.raises(sdbg.SdbgError) as ei:
        gpu_count(rs, 21, 2, False, prefix_len=0, mem_budget=1000)
    assert ei.value.code == -3


def test_empty_and_degenerate_inputs():
    cases = [[], ["ACG"], ["NNNNNNNN", "AC"], ["acgtacgtNacgtacgt"], ["A" * 300], ["AC" * 100, "ACGT" * 10]]
    for reads in cases:
        for k, d, mercy in [(3, 1, False), (3, 2, True), (5, 2, True)]:
            rs = synth.from_strings(reads, k, d, mercy)
            rs.name = f"{reads[:1]}"
            _parity(rs, k, d, mercy)


def test_single_huge_run_of_equal_keys():
    """All reads identical and low-complexity: a few keys with huge counts
    (buckets of equal keys longer than a leaf)."""
    rs = synth.from_strings(["A" * 150] * 4000 + ["ACGTTGCA" * 20] * 1000, 31)
    _parity(rs, 31, 2, True)
    _parity(rs, 31, 5000, False)


def test_build_from_host_edges():
    rs = synth.random_small(100, 20, 60, 300, 0.03, 9)
    o = oracle.count_solid(rs.seq, rs.offsets, 9, 2, True)
    e = sdbg.edges_from_host(o.keys, o.counts, 9)
    h = gpu_graph(e)
    assert_graph_equal(h, oracle.build_graph(o.keys, o.counts, 9))
    # a non-RC-closed edge set (half of the edges) is still a valid input
    half = slice(0, None, 2)
    e2 = sdbg.edges_from_host(o.keys[half], o.counts[half], 9)
    assert_graph_equal(gpu_graph(e2), oracle.build_graph(o.keys[half], o.counts[half], 9))


def test_build_rejects_unsorted_edges():
    keys = np.array([[5], [3]], dtype=np.uint64)
    e = sdbg.edges_from_host(keys, np.array([2, 2], dtype=np.uint32), 3)
    with pytest.raises(sdbg.SdbgError):
        sdbg.build(e)


def test_repeat_calls_are_deterministic():
    rs = synth.tiny(scale=0.3)
    outs = []
    for _ in range(3):
        e, keys, cnt = gpu_count(rs, 21, 2, True)
        outs.append((keys, cnt, gpu_graph(e)))
    for keys, cnt, h in outs[1:]:
        assert np.array_equal(keys, outs[0][0]) and np.array_equal(cnt, outs[0][1])
        assert_graph_equal(h, outs[0][2])


def test_three_word_keys_mercy_repeatable():
    """Regression: mercy lookups with 3-word keys (k = 64..95) must be exact
    on every run (they once varied between runs on the device)."""
    rs = synth.metagenome_long(scale=0.0015, k=81)
    o = oracle.count_solid(rs.seq, rs.offsets, 81, 2, True)
    for rep in range(3):
        say(f"repeat {rep}")
        e, keys, cnt = gpu_count(rs, 81, 2, True)
        assert e.n_mercy == o.n_mercy
        assert np.array_equal(keys, o.keys) and np.array_equal(cnt, o.counts)


@pytest.mark.parametrize("k", [5, 21, 31, 41])
def test_mercy_lookup_table_overfull_paths(k):
    """A mercy lookup table 4x, 32x and 256x smaller than it is sized for
    (mercy_shift): more and more buckets hold more entries than slots, and
    at 256x whole fill blocks overflow their LDS stage, so lookups take the
    sorted-set path; results must not change."""
    if k < 8:
        rs = synth.random_small(300, k, k + 60, 200, 0.05, 42)
    else:
        rs = synth.metagenome_long(scale=0.0015, k=k)
    o = oracle.count_solid(rs.seq, rs.offsets, k, 2, True)
    assert o.n_mercy > 0
    try:
        for shift in (2, 5, 8):
            say(f"k={k} mercy_shift={shift}")
            sdbg.tune_set({"mercy_shift": shift})
            e, keys, cnt = gpu_count(rs, k, 2, True)
            assert e.n_mercy == o.n_mercy
            assert np.array_equal(keys, o.keys) and np.array_equal(cnt, o.counts)
    finally:
        sdbg.tune_set(None)


@pytest.mark.parametrize("k,copies", [(31, 2100), (81, 1100), (99, 1100)])
@pytest.mark.parametrize("cap_shift", [0, 1])
def test_many_copies_of_one_read(k, copies, cap_shift):
    """One 150 bp read repeated a little more often than a leaf holds (an
    amplicon or spike-in), plus random reads: every window of that read is a
    key whose run is longer than a leaf, so the partition must isolate the
    run without cutting one digit per level through all 2(k+1) key bits."""
    rng = np.random.Generator(np.random.PCG64([0x14097208, 99, k, copies]))
    read = "".join("ACGT"[c] for c in rng.integers(0, 4, 150))
    rs_bg = synth.random_small(400, k + 1, k + 60, 3000, 0.02, 7 + k)
    reads = [r.decode() for r in rs_bg.reads()] + [read] * copies
    rs = synth.from_strings(reads, k, 2, True)
    rs.name = f"{copies} copies of one read"
    try:
        sdbg.tune_set({"leaf_cap_shift": cap_shift})
        _parity(rs, k, 2, True)
    finally:
        sdbg.tune_set(None)


def test_device_offsets_must_not_decrease():
    """Device-resident offsets are validated like host ones: a decreasing
    pair is an argument error, before any read is touched."""
    import torch

    seq = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for offs in ([0, 40, 10, 64], [0, 64, 63], [0, 1 << 40, 100]):
        off = torch.tensor(offs, dtype=torch.int64, device="cuda")
        with pytest.raises(sdbg.SdbgError) as ei:
            sdbg.count_solid(seq, off, 5, 2, True)
        assert ei.value.code == -1 and "non-decreasing" in str(ei.value)
