"""TEST INFRASTRUCTURE ONLY: multiple k with contig feedback.

Section 2 (fourth paragraph) and Fig. 1 describe the workflow: graphs are
built from a small k to a large one, each is cleaned, and the contigs of one
k go into the graph of the next.  The paper does not say how contigs enter
the next graph; the reading fixed for the device path: for each k in
ascending order,

1. E = the solid edges of the reads (count_solid with d and mercy);
2. from the second k on, every (k+1)-mer of the previous k's unitigs, on
   both strands, joins E with its count of occurrences in them (count_solid
   of the unitigs with d = 1, no mercy), counts of keys in both summed;
3. tips of at most tip_factor * k edges are removed (oracle/tips.py), then
   bubbles of unitigs of at most bubble_factor * k edges and then unitigs
   of at most low_cov_factor * k edges below low_cov_permille / 1000 of
   their neighbours' mean multiplicity (oracle/cleaning.py; a factor of 0
   skips the step);
4. the unitigs of the remaining edges are taken (oracle/unitigs.py).

Composes the oracle's own pieces; nothing here comes from the device path.
"""

from __future__ import annotations

import numpy as np

from . import count_solid
from .cleaning import bubbles, low_coverage
from .tips import key_to_edge, removed_tips
from .unitigs import unitigs


def _union(a_keys, a_cnt, b_keys, b_cnt):
    """Keys of either set (n x w arrays of words, most significant first),
    counts summed, ascending."""
    w = np.asarray(a_keys).shape[1]
    tot: dict[tuple, int] = {}
    for keys, cnt in ((a_keys, a_cnt), (b_keys, b_cnt)):
        for row, c in zip(np.asarray(keys, dtype=np.uint64), cnt):
            t = tuple(int(x) for x in row)
            tot[t] = tot.get(t, 0) + int(c)
    order = sorted(tot)  # tuples of words compare as the numbers they spell
    return np.array(order, dtype=np.uint64).reshape(len(order), w), np.array([tot[t] for t in order], dtype=np.uint64)


def multi_k(seq, offsets, ks, d: int = 2, mercy: bool = True, tip_factor: int = 2, bubble_factor: int = 0,
            low_cov_factor: int = 0, low_cov_permille: int = 0):
    """Returns (the last k's unitigs as (first edge, edges, multiplicity,
    sequence) tuples, per-k stats [edges, edges added by the unitigs, edges
    removed as tips, in bubbles and for low coverage, unitigs])."""
    prev = None
    stats = []
    res = []
    for k in ks:
        e = count_solid(seq, offsets, k, d, mercy)
        keys, cnt = e.keys, e.counts.astype(np.uint64)
        n_read = len(cnt)
        if prev is not None and len(prev[1]) > 1:
            ce = count_solid(prev[0], prev[1], k, 1, False)
            keys, cnt = _union(keys, cnt, ce.keys, ce.counts)
        edges = [key_to_edge(row, k) for row in np.asarray(keys, dtype=np.uint64).reshape(len(cnt), -1)]
        gone = removed_tips(edges, tip_factor * k) if tip_factor else set()
        valid = [x not in gone for x in edges]
        n_bub = n_low = 0
        if bubble_factor:
            b = bubbles(edges, cnt, valid, k, bubble_factor * k)
            valid = [ok and x not in b for x, ok in zip(edges, valid)]
            n_bub = len(b)
        if low_cov_factor:
            lo = low_coverage(edges, cnt, valid, k, low_cov_factor * k, low_cov_permille)
            valid = [ok and x not in lo for x, ok in zip(edges, valid)]
            n_low = len(lo)
        res = unitigs(edges, cnt, valid)
        stats.append([len(edges), len(edges) - n_read, len(gone), n_bub, n_low, len(res)])
        text = "".join(r[3] for r in res).encode()
        off = np.zeros(len(res) + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(r[3]) for r in res])
        prev = (np.frombuffer(text, dtype=np.uint8).copy(), off)
    return res, np.array(stats, dtype=np.uint64)
