"""Bubble merging and low-local-coverage removal on the device
(sdbg_merge_bubbles, sdbg_remove_low_coverage) against the oracle on the
explicit graph (oracle/cleaning.py): the hand-built graphs of
tests/test_cleaning_oracle.py, and seeded workloads cleaned in sequence
(tips, then bubbles, then low local coverage, unitigs taken again before
each step), edge by edge.  The oracle's edges come from the oracle's own
count; the device's edge set equals it (checked first), so the i-th real row
of the device graph is the oracle's i-th edge."""

from __future__ import annotations

import random

import numpy as np
import pytest

import brute
import oracle
from gpu_util import bits, gpu_count, say
from oracle import cleaning, tips
from paper_1409_7208_amd import sdbg, synth
from test_cleaning_oracle import _bubble
from test_tips_oracle import K, edges_of, main_path, rand_seq

pytestmark = pytest.mark.gpu


class Cleaner:
    """A device graph with its index; valid() = the valid mask over E."""

    def __init__(self, e: sdbg.Edges):
        self.g = sdbg.build(e)
        self.ix = sdbg.Index(self.g)
        h = self.g.to_host()
        self.real = ((h.W & 7) != 0) & ~bits(h.tip, h.m)

    def valid(self) -> np.ndarray:
        h = self.g.to_host()
        return bits(h.valid, h.m)[self.real]

    def step(self, what: str, *args) -> int:
        if what == "tips":
            return self.ix.remove_tips(*args)
        u = self.ix.unitigs()
        n = self.ix.merge_bubbles(u, *args) if what == "bubbles" else self.ix.remove_low_coverage(u, *args)
        u.close()
        return n

    def close(self):
        self.ix.close()
        self.g.close()


def _oracle_step(what, edges, counts, valid, k, *args):
    if what == "tips":  # tips are found on the graph as built
        gone = tips.removed_tips(edges, *args)
    elif what == "bubbles":
        gone = cleaning.bubbles(edges, counts, valid, k, *args)
    else:
        gone = cleaning.low_coverage(edges, counts, valid, k, *args)
    return valid & ~np.array([x in gone for x in edges])


def _hand(E, cnt):
    edges = sorted(E, key=brute.edge_key)
    c = [cnt[x] for x in edges]
    keys = np.array([brute.key_to_words(brute.edge_key(x), K) for x in edges], dtype=np.uint64)
    return edges, c, sdbg.edges_from_host(keys, np.array(c, dtype=np.uint32), K)


def test_cleaning_of_hand_built_graphs():
    rng = random.Random(31)
    s = main_path(rng)
    alt = _bubble(rng, s)
    a2 = _bubble(rng, s)
    branch_in = rand_seq(3, rng, last_not=s[39]) + s[40 : 40 + K]
    branch_out = s[35 : 35 + K] + rand_seq(4, rng, first_not=s[35 + K])
    cases = [
        ({x: 10 for x in edges_of(s)} | {x: 2 for x in edges_of(alt)}, [("bubbles", 20)]),
        ({x: 5 for x in edges_of(s, alt)}, [("bubbles", 20)]),
        ({x: 10 for x in edges_of(s)} | {x: 2 for x in edges_of(alt)}, [("bubbles", K + 3), ("bubbles", K + 4)]),
        ({x: 3 for x in edges_of(s)} | {x: 9 for x in edges_of(alt)} | {x: 4 for x in edges_of(a2)},
         [("bubbles", 20)]),
        ({x: 20 for x in edges_of(s)} | {x: 1 for x in edges_of(branch_in)},
         [("low", 10, 50), ("low", 10, 51), ("low", 2, 900)]),
        ({x: 20 for x in edges_of(s)} | {x: 15 for x in edges_of(branch_out)}, [("low", 10, 200), ("low", 10, 800)]),
        ({x: 10 for x in edges_of(s)} | {x: 1 for x in edges_of(alt)}, [("low", 20, 100), ("low", 20, 150)]),
        ({x: 1 for x in edges_of(main_path(rng, n=K + 4))}, [("low", 10, 900)]),
    ]
    for cnt, steps in cases:
        edges, c, e = _hand(cnt.keys(), cnt)
        for step in steps:
            cl = Cleaner(e)  # each step on a fresh graph
            want = _oracle_step(step[0], edges, c, np.ones(len(edges), dtype=bool), K, *step[1:])
            n = cl.step(*step)
            got = cl.valid()
            assert np.array_equal(got, want), step
            assert n == int((~want).sum())
            cl.close()
        e.close()


@pytest.mark.parametrize("case", [
    ("tiny", 21, False, 1.0),
    ("metagenome", 31, True, 0.002),
    ("metagenome", 41, True, 0.002),
    ("metagenome", 81, True, 0.002),
])
def test_cleaning_of_workload_graphs(case):
    name, k, mercy, scale = case
    rs = synth.tiny(scale) if name == "tiny" else synth.metagenome(scale, k=k)
    oe = oracle.count_solid(rs.seq, rs.offsets, k, 2, mercy)
    edges = [tips.key_to_edge(row, k) for row in np.asarray(oe.keys, dtype=np.uint64).reshape(len(oe.counts), -1)]
    e, keys, _ = gpu_count(rs, k, 2, mercy)
    assert np.array_equal(keys, oe.keys)
    cl = Cleaner(e)
    e.close()
    valid = np.ones(len(edges), dtype=bool)
    for step in (("tips", 2 * k), ("bubbles", 2 * k), ("low", 2 * k, 200), ("bubbles", 4 * k), ("low", 4 * k, 900)):
        want = _oracle_step(step[0], edges, oe.counts, valid, k, *step[1:])
        n = cl.step(*step)
        got = cl.valid()
        say(f"{name} k={k} {step}: {int(valid.sum() - want.sum())} edges removed (device {n})")
        assert np.array_equal(got, want), step
        assert n == int(valid.sum() - want.sum())
        valid = want
    cl.close()
