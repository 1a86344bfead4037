"""Tip removal on the device (sdbg_remove_tips) against the oracle's tip
removal on the explicit graph (oracle/tips.py): the hand-built graphs of
tests/test_tips_oracle.py, and the graphs of seeded workloads (one to three
key words, mercy on and off), edge by edge.  The oracle's edges come from
the oracle's own count; the device's edge set equals it (checked first), so
the i-th real row of the device graph is the oracle's i-th edge."""

from __future__ import annotations

import random

import numpy as np
import pytest

import brute
import oracle
from gpu_util import gpu_count, say
from oracle import tips
from paper_1409_7208_amd import sdbg, synth
from test_tips_oracle import K, edges_of, main_path, rand_seq

pytestmark = pytest.mark.gpu


def _bits(words: np.ndarray, m: int) -> np.ndarray:
    return np.unpackbits(words.view(np.uint8), bitorder="little")[:m].astype(bool)


def _device_removed(e: sdbg.Edges, max_len: int):
    """Build the graph of e, remove its tips; the removed mask over E (in
    key order), the count the call reported, and a second call's count."""
    g = sdbg.build(e)
    before = g.to_host()
    ix = sdbg.Index(g)
    n = ix.remove_tips(max_len)
    after = g.to_host()
    n2 = ix.remove_tips(max_len)  # validity is not read: nothing new to clear
    again = g.to_host()
    ix.close()
    g.close()
    assert np.array_equal(after.valid, again.valid)
    vb, va = _bits(before.valid, before.m), _bits(after.valid, after.m)
    assert not (va & ~vb).any()
    return vb[vb] & ~va[vb], n, n2


def test_tips_of_hand_built_graphs():
    rng = random.Random(11)
    s = main_path(rng)
    graphs = [
        edges_of(s, rand_seq(3, rng, last_not=s[39]) + s[40 : 40 + K]),  # branch joining
        edges_of(s, s[35 : 35 + K] + rand_seq(4, rng, first_not=s[35 + K])),  # branch leaving
        edges_of(main_path(rng, n=K + 3)),  # isolated short path
        edges_of(s, s[30 : 30 + K] + rand_seq(4, rng, first_not=s[30 + K], last_not=s[30 + K + 3])
                 + s[30 + K + 4 : 30 + 2 * K + 4]),  # bubble
    ]
    for E in graphs:
        edges = sorted(E, key=brute.edge_key)
        keys = np.array([brute.key_to_words(brute.edge_key(x), K) for x in edges], dtype=np.uint64)
        e = sdbg.edges_from_host(keys, np.full(len(edges), 2, dtype=np.uint32), K)
        for max_len in (2, 3, 10):
            want = np.array([x in tips.removed_tips(edges, max_len) for x in edges])
            got, n, n2 = _device_removed(e, max_len)
            assert np.array_equal(got, want), (max_len, edges)
            assert n == int(want.sum()) and n2 == 0
        e.close()


@pytest.mark.parametrize("case", [
    ("tiny", 21, False, 1.0),
    ("metagenome", 31, True, 0.002),
    ("metagenome", 41, True, 0.002),
    ("metagenome", 81, True, 0.002),
])
def test_tips_of_workload_graphs(case):
    name, k, mercy, scale = case
    rs = synth.tiny(scale) if name == "tiny" else synth.metagenome(scale, k=k)
    max_len = 2 * k
    oe = oracle.count_solid(rs.seq, rs.offsets, k, 2, mercy)
    want = tips.removed_mask(oe.keys, k, max_len)
    e, keys, _ = gpu_count(rs, k, 2, mercy)
    assert np.array_equal(keys, oe.keys)
    got, n, n2 = _device_removed(e, max_len)
    e.close()
    say(f"{name} k={k}: {len(keys)} edges, {int(want.sum())} in tips of at most {max_len} edges")
    assert np.array_equal(got, want)
    assert n == int(want.sum()) and n2 == 0


def test_remove_tips_rejects_an_index_of_another_graph():
    rs = synth.tiny(0.05)
    e, _, _ = gpu_count(rs, 21, 2, False)
    g1, g2 = sdbg.build(e), sdbg.build(e)
    ix = sdbg.Index(g1)
    ix._graph = g2  # the call gets g2 with g1's index
    with pytest.raises(sdbg.SdbgError):
        ix.remove_tips(42)
    ix._graph = g1
    ix.close()
    g1.close()
    g2.close()
    e.close()
