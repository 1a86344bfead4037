"""Identities the device path relies on, checked on the oracle's output (no
GPU).

* Counting on one strand: an edge's count over both strands equals the
  number of windows whose canonical key (the smaller of a window's two
  strands' keys) it is, a window that is its own reverse complement counting
  twice (Section 2, third paragraph, with both strands counted).
* Node sets: a window is solid exactly when its last base is in the
  out-set of its source k-mer, and exactly when its first base is in the
  in-set of its target k-mer; its mercy dead-end flags are empty sets of
  those k-mers (no solid edge out of the target, none into the source).

Everything here is written from the definitions on strings, independently
of the oracle's code."""

from __future__ import annotations

import collections

import pytest

import oracle
from paper_1409_7208_amd import synth

CODE = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def _rc(s: str) -> str:
    return "".join(COMP[c] for c in reversed(s))


def _key(e: str) -> int:
    """Edge key of the (k+1)-mer e: digits e[k-1], ..., e[0], e[k]."""
    k = len(e) - 1
    v = 0
    for i in range(k - 1, -1, -1):
        v = 4 * v + CODE[ord(e[i])]
    return 4 * v + CODE[ord(e[k])]


def _windows(rs, k: int):
    for r in rs.reads():
        s = r.decode().upper()
        for j in range(len(s) - k):
            w = s[j : j + k + 1]
            if set(w) <= set("ACGT"):
                yield w


def _solid(rs, k: int, d: int) -> dict[int, int]:
    e = oracle.count_solid(rs.seq, rs.offsets, k, d, False)
    return {int(x): int(c) for x, c in zip(e.keys[:, -1], e.counts)}


@pytest.mark.parametrize("k,seed", [(3, 1), (4, 2), (7, 3), (8, 4), (15, 5), (21, 6), (31, 7)])
def test_canonical_count_equals_both_strand_count(k, seed):
    rs = synth.random_small(80, k + 1, k + 50, 300, 0.03, 4000 + seed, n_rate=0.01)
    canon = collections.Counter()
    for w in _windows(rs, k):
        r = _rc(w)
        c = min(_key(w), _key(r))
        canon[c] += 2 if w == r else 1
    got = _solid(rs, k, 1)  # every edge, with its count over both strands
    assert len(got) > 0
    for x, cnt in got.items():
        # decode the key back to its (k+1)-mer to find its reverse complement
        digits = [(x >> (2 * (i + 1))) & 3 for i in range(k)] + [x & 3]
        s = "".join("ACGT"[v] for v in digits)
        cx = min(x, _key(_rc(s)))
        assert canon[cx] == cnt, (s, canon[cx], cnt)
    # and nothing is counted that the oracle does not have
    for cx, n in canon.items():
        assert got.get(cx) == n


@pytest.mark.parametrize("k,seed", [(5, 11), (11, 12), (21, 13), (31, 14)])
def test_node_sets_give_solidity_and_dead_ends(k, seed):
    rs = synth.random_small(120, k + 1, k + 60, 400, 0.02, 5000 + seed)
    solid = _solid(rs, k, 2)
    edges = set()
    for x in solid:
        digits = [(x >> (2 * (i + 1))) & 3 for i in range(k)] + [x & 3]
        edges.add("".join("ACGT"[v] for v in digits))
    out_set = collections.defaultdict(set)  # k-mer -> last bases of solid edges out of it
    in_set = collections.defaultdict(set)  # k-mer -> first bases of solid edges into it
    for e in edges:
        out_set[e[:k]].add(e[k])
        in_set[e[1:]].add(e[0])
    n_solid = 0
    for w in _windows(rs, k):
        src, tgt = w[:k], w[1:]
        is_solid = w in edges
        n_solid += is_solid
        assert is_solid == (w[k] in out_set[src]) == (w[0] in in_set[tgt])
        if is_solid:
            # dead-end flags from their definitions on the solid set ...
            no_out = not any(e[:k] == tgt for e in edges)
            no_in = not any(e[1:] == src for e in edges)
            # ... are the empty sets of the window's end k-mers
            assert no_out == (len(out_set[tgt]) == 0)
            assert no_in == (len(in_set[src]) == 0)
    assert n_solid > 0
