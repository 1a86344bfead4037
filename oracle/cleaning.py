"""TEST INFRASTRUCTURE ONLY: bubble merging and low-local-coverage removal
on the explicit de Bruijn graph.

Section 2 (fourth paragraph) lists them, with tip removal, as the cleaning
of each graph, and notes that removing low local coverage edges suits the
uneven depth of metagenomes; it defines neither.  The readings fixed for the
device path, on the unitigs of the valid edges (oracle/unitigs.py), where a
unitig u of len(u) edges runs from its start node s(u) (the source of its
first edge) to its end node t(u) (the target of its last edge), has
multiplicity mult(u), and cycles take part in neither step:

* bubbles: unitigs of at most max_len edges that share both s and t form a
  group; in a group of two or more, every unitig but the one of highest mean
  multiplicity (mult / len, compared as mult(a) * len(b) against
  mult(b) * len(a); ties to the smaller first edge) is removed;
* low local coverage: for a unitig u of at most max_len edges, its
  neighbouring edges are the valid edges other than u's first and last edge
  that leave or enter s(u) or t(u); if there is at least one and
  mult(u) * count * 1000 < ratio_permille * len(u) * sum of their counts (the
  mean multiplicity of u below ratio_permille / 1000 of the neighbours'
  mean), every edge of u is removed.

Each step decides on the graph as given and removes all its unitigs at once.
Plain Python over strings; returns the set of removed edges.
"""

from __future__ import annotations

from collections import defaultdict

from .unitigs import unitigs


def _unitig_edges(seq: str, n: int, k: int) -> list[str]:
    return [seq[i : i + k + 1] for i in range(n)]


def _is_cycle(seq: str, k: int, n_in, n_out) -> bool:
    s = seq[:k]
    return n_in[s] == 1 and n_out[s] == 1  # a non-cycle unitig starts at a branching node


def _degrees(edges, valid):
    n_in, n_out = defaultdict(int), defaultdict(int)
    for x, ok in zip(edges, valid):
        if ok:
            n_out[x[:-1]] += 1
            n_in[x[1:]] += 1
    return n_in, n_out


def bubbles(edges: list[str], counts, valid, k: int, max_len: int) -> set[str]:
    n_in, n_out = _degrees(edges, valid)
    groups = defaultdict(list)
    for first, n, mult, seq in unitigs(edges, counts, valid):
        if n <= max_len and not _is_cycle(seq, k, n_in, n_out):
            groups[(seq[:k], seq[-k:])].append((first, n, mult, seq))
    gone: set[str] = set()
    for g in groups.values():
        if len(g) < 2:
            continue
        best = g[0]
        for u in g[1:]:
            a, b = u[2] * best[1], best[2] * u[1]  # mean of u against mean of best
            if a > b or (a == b and u[0] < best[0]):
                best = u
        for u in g:
            if u is not best:
                gone.update(_unitig_edges(u[3], u[1], k))
    return gone


def low_coverage(edges: list[str], counts, valid, k: int, max_len: int, ratio_permille: int) -> set[str]:
    n_in, n_out = _degrees(edges, valid)
    out_e, in_e = defaultdict(list), defaultdict(list)
    cnt = {}
    for x, c, ok in zip(edges, counts, valid):
        if ok:
            out_e[x[:-1]].append(x)
            in_e[x[1:]].append(x)
            cnt[x] = int(c)
    gone: set[str] = set()
    for first, n, mult, seq in unitigs(edges, counts, valid):
        if n > max_len or _is_cycle(seq, k, n_in, n_out):
            continue
        own = _unitig_edges(seq, n, k)
        s, t = seq[:k], seq[-k:]
        nb = set()
        for v in {s, t}:
            nb.update(out_e[v])
            nb.update(in_e[v])
        nb -= {own[0], own[-1]}
        if not nb:
            continue
        total = sum(cnt[x] for x in nb)
        if mult * len(nb) * 1000 < ratio_permille * n * total:
            gone.update(own)
    return gone
