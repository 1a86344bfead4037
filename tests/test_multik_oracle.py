"""Pins of the multi-k oracle (oracle/multik.py).  The case the workflow is
for: reads that overlap by more than a small k but less than a large one.
At the large k alone the graph falls apart between reads; with the small
k's contig fed in, the large-k graph holds the whole genome again, and the
edges the contig adds are exactly the (k+1)-mers that span the read
junctions.  Also: one k alone is the plain count, tip removal and unitigs."""

from __future__ import annotations

import random

import numpy as np

import brute
import oracle
from oracle import cleaning, multik, tips
from oracle import unitigs as U


def _genome(rng, n):
    while True:  # no repeated 15-mer on either strand
        g = "".join(rng.choice("ACGT") for _ in range(n))
        both = g + "N" + brute.revcomp(g)
        kms = [both[i : i + 15] for i in range(len(both) - 14) if "N" not in both[i : i + 15]]
        if len(set(kms)) == len(kms):
            return g


def _reads(g, length=40, step=15):
    rs = [g[i : i + length] for i in range(0, len(g) - length + 1, step)]
    if (len(g) - length) % step:
        rs.append(g[-length:])
    seq = np.frombuffer("".join(rs).encode(), dtype=np.uint8).copy()
    off = np.zeros(len(rs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(r) for r in rs])
    return rs, seq, off


def test_contigs_bridge_reads_at_the_larger_k():
    rng = random.Random(3)
    g = _genome(rng, 300)
    rs, seq, off = _reads(g)  # neighbours overlap by 25 bases
    alone, _ = multik.multi_k(seq, off, [31], d=1, mercy=False, tip_factor=0)
    assert len(alone) > 2  # 32-mers never span two reads: pieces only
    # (with tip removal, each piece, an isolated path of 9 edges, would go)
    assert multik.multi_k(seq, off, [31], d=1, mercy=False)[0] == []
    res, st = multik.multi_k(seq, off, [15, 31], d=1, mercy=False)
    assert sorted(r[3] for r in res) == sorted([g, brute.revcomp(g)])
    # the contig adds the 32-mers of g (both strands) that no read holds
    in_reads = {r[i : i + 32] for r in rs for i in range(len(r) - 31)}
    span = {g[i : i + 32] for i in range(len(g) - 31)} - in_reads
    assert int(st[1, 1]) == 2 * len(span) > 0
    assert int(st[1, 0]) == 2 * (len(g) - 31)
    # multiplicity: read occurrences plus two from the contigs (g itself and
    # the other strand of its reverse complement, both unitigs at k = 15)
    want_mult = sum(sum(1 for r in rs for i in range(len(r) - 31) if r[i : i + 32] == x) + 2
                    for x in {g[i : i + 32] for i in range(len(g) - 31)})
    fwd = [r for r in res if r[3] == g][0]
    assert fwd[2] == want_mult


def test_single_k_is_count_tips_unitigs():
    rng = random.Random(4)
    g = _genome(rng, 400)
    reads = []
    for _ in range(150):  # random reads with an error now and then
        i = rng.randrange(0, len(g) - 50)
        r = list(g[i : i + 50])
        if rng.random() < 0.2:
            r[rng.randrange(50)] = rng.choice("ACGT")
        reads.append("".join(r))
    seq = np.frombuffer("".join(reads).encode(), dtype=np.uint8).copy()
    off = np.zeros(len(reads) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(r) for r in reads])
    k = 21
    res, st = multik.multi_k(seq, off, [k], d=2, mercy=True, tip_factor=2)
    e = oracle.count_solid(seq, off, k, 2, True)
    edges = [tips.key_to_edge(row, k) for row in e.keys]
    gone = tips.removed_tips(edges, 2 * k)
    assert res == U.unitigs(edges, e.counts, [x not in gone for x in edges])
    assert st.tolist() == [[len(edges), 0, len(gone), 0, 0, len(res)]]
    # with bubbles and low coverage: tips, then bubbles, then low coverage
    res2, st2 = multik.multi_k(seq, off, [k], 2, True, 2, 2, 2, 400)
    valid = [x not in gone for x in edges]
    b = cleaning.bubbles(edges, e.counts, valid, k, 2 * k)
    valid = [ok and x not in b for x, ok in zip(edges, valid)]
    lo = cleaning.low_coverage(edges, e.counts, valid, k, 2 * k, 400)
    valid = [ok and x not in lo for x, ok in zip(edges, valid)]
    assert res2 == U.unitigs(edges, e.counts, valid)
    assert st2.tolist() == [[len(edges), 0, len(gone), len(b), len(lo), len(res2)]]
