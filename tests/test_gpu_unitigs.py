"""Unitigs on the device (sdbg_unitigs_build) against the unitig oracle on
the explicit graph (oracle/unitigs.py): the hand-built graphs of
tests/test_unitigs_oracle.py (paths, branches, a bubble, cycles, a
self-loop, removed edges) and seeded workloads before and after tip
removal, unitig by unitig (first edge, length, multiplicity, sequence).
The oracle's edges come from the oracle's own count; the device's edge set
equals it (checked first), so the i-th real row of the device graph is the
oracle's i-th edge.  Last, the unitigs of one k are counted as a device read
set at a larger k and compared with the oracle's count of the same
sequences."""

from __future__ import annotations

import random

import numpy as np
import pytest

import brute
import oracle
from gpu_util import bits, gpu_count, say
from oracle import tips
from oracle import unitigs as U
from paper_1409_7208_amd import sdbg, synth
from test_tips_oracle import K, edges_of, main_path, rand_seq

pytestmark = pytest.mark.gpu


def _device_unitigs(e: sdbg.Edges, tip_len: int = 0):
    """Build, optionally remove tips, take the unitigs; returns the host
    unitigs with first_row mapped to the index of the edge in E."""
    g = sdbg.build(e)
    ix = sdbg.Index(g)
    if tip_len:
        ix.remove_tips(tip_len)
    u = ix.unitigs()
    h = g.to_host()
    hu = u.to_host()
    u.close()
    ix.close()
    g.close()
    real = np.flatnonzero(((h.W & 7) != 0) & ~bits(h.tip, h.m))
    idx = np.searchsorted(real, hu.first_row)
    assert np.array_equal(real[idx], hu.first_row)
    return [(int(idx[i]), int(hu.len[i]), int(hu.mult[i]), hu.sequence(i)) for i in range(len(idx))], hu


def _compare(got, want):
    assert len(got) == len(want)
    for a, b in zip(got, want):
        assert a == b, (a, b)


def _hand_graph(E, counts=None):
    edges = sorted(E, key=brute.edge_key)
    cnt = [counts[x] if counts else 1 + brute.edge_key(x) % 5 for x in edges]
    keys = np.array([brute.key_to_words(brute.edge_key(x), K) for x in edges], dtype=np.uint64)
    e = sdbg.edges_from_host(keys, np.array(cnt, dtype=np.uint32), K)
    return edges, cnt, e


def _cycle(rng, n=30):
    while True:
        c = rand_seq(n, rng)
        c2 = c + c[:K]
        kms = [c2[i : i + K] for i in range(n)]
        if len(set(kms)) == n:
            return {c2[i : i + K + 1] for i in range(n)}


def test_unitigs_of_hand_built_graphs():
    rng = random.Random(21)
    s = main_path(rng)
    p, q = 30, 30 + K + 4
    graphs = [
        edges_of(s),
        edges_of(s, rand_seq(3, rng, last_not=s[39]) + s[40 : 40 + K]),  # branch joining
        edges_of(s, s[35 : 35 + K] + rand_seq(4, rng, first_not=s[35 + K])),  # branch leaving
        edges_of(s, s[p : p + K] + rand_seq(4, rng, first_not=s[p + K], last_not=s[q - 1]) + s[q : q + K]),  # bubble
        _cycle(rng),
        _cycle(rng, 12) | edges_of(main_path(rng, n=40)),  # a cycle next to a path
        {"A" * (K + 1)},  # self-loop
        {"A" * (K + 1), "C" * (K + 1), "G" * (K + 1)} | _cycle(rng, 9),
    ]
    for E in graphs:
        edges, cnt, e = _hand_graph(E)
        want = U.unitigs(edges, cnt, [True] * len(edges))
        got, hu = _device_unitigs(e)
        _compare(got, want)
        e.close()


def test_unitigs_after_tip_removal_of_hand_built_graph():
    rng = random.Random(22)
    s = main_path(rng)
    branch = rand_seq(3, rng, last_not=s[39]) + s[40 : 40 + K]
    edges, cnt, e = _hand_graph(edges_of(s, branch))
    gone = tips.removed_tips(edges, 10)
    want = U.unitigs(edges, cnt, [x not in gone for x in edges])
    assert [w[3] for w in want] == [s]
    got, _ = _device_unitigs(e, tip_len=10)
    _compare(got, want)
    e.close()


@pytest.mark.parametrize("case", [
    ("tiny", 21, False, 1.0, 0),
    ("tiny", 21, False, 1.0, 42),
    ("metagenome", 31, True, 0.002, 62),
    ("metagenome", 41, True, 0.002, 0),
    ("metagenome", 81, True, 0.002, 162),
])
def test_unitigs_of_workload_graphs(case):
    name, k, mercy, scale, tip_len = case
    rs = synth.tiny(scale) if name == "tiny" else synth.metagenome(scale, k=k)
    oe = oracle.count_solid(rs.seq, rs.offsets, k, 2, mercy)
    edges = [tips.key_to_edge(row, k) for row in np.asarray(oe.keys, dtype=np.uint64).reshape(len(oe.counts), -1)]
    valid = ~tips.removed_mask(oe.keys, k, tip_len) if tip_len else np.ones(len(edges), dtype=bool)
    want = U.unitigs(edges, oe.counts, valid)
    e, keys, _ = gpu_count(rs, k, 2, mercy)
    assert np.array_equal(keys, oe.keys)
    got, hu = _device_unitigs(e, tip_len)
    e.close()
    say(f"{name} k={k} tips<={tip_len}: {len(edges)} edges, {len(want)} unitigs, "
        f"longest {max(w[1] for w in want)} edges, {hu.n_cycles} cycles")
    _compare(got, want)


def test_unitigs_counted_at_the_next_k():
    """Unitigs as a device read set (the feedback of one k into the next)."""
    rs = synth.metagenome(0.002, k=21)
    e, _, _ = gpu_count(rs, 21, 2, True)
    g = sdbg.build(e)
    ix = sdbg.Index(g)
    ix.remove_tips(42)
    u = ix.unitigs()
    hu = u.to_host()
    k2 = 41
    e2 = sdbg.count_solid(u.as_reads(), None, k2, 1, False)
    keys2, cnt2 = e2.to_host()
    want = oracle.count_solid(hu.seq, hu.offsets, k2, 1, False)
    assert np.array_equal(keys2, want.keys) and np.array_equal(cnt2, want.counts)
    say(f"{hu.len.size} unitigs, {hu.seq.size} bases -> {len(cnt2)} edges at k={k2}")
    for x in (e2, u, ix, g, e):
        x.close()
