"""TEST INFRASTRUCTURE ONLY: tip removal on the explicit de Bruijn graph.

Section 2 (fourth paragraph) names tip removal as one of the cleaning steps
applied to each graph; the paper gives no definition, so this follows the
reading fixed for the device path: on the graph as built (all edges, solid
and mercy), with degrees counted over its edges,

* a forward tip is a path v0 -> v1 -> ... -> vj of j >= 1 edges with
  indeg(v0) = 0, outdeg(vi) = 1 for i < j, indeg(vi) = 1 for 0 < i < j, that
  ends at a node vj with indeg(vj) >= 2 (it joins the graph) or
  outdeg(vj) = 0 (an isolated path);
* a backward tip is the mirror image: vj -> ... -> v1 -> v0 with
  outdeg(v0) = 0, indeg(vi) = 1 for i < j, outdeg(vi) = 1 for 0 < i < j,
  ending (walking backwards) at vj with outdeg(vj) >= 2 or indeg(vj) = 0;
* every edge of every tip with j <= max_len is removed, all at once (tips
  are found on the original graph, so removing one does not create another
  in the same pass).

Plain Python over strings: nodes are k-mers, an edge (k+1)-mer x goes from
x[0..k-1] to x[1..k].  Slow, for test-sized graphs.
"""

from __future__ import annotations

from collections import defaultdict

import numpy as np

_BASES = "ACGT"


def key_to_edge(words, k: int) -> str:
    """The (k+1)-mer of an edge key (digits e[k-1], ..., e[0], e[k] of the
    base-4 number; words most significant first)."""
    key = 0
    for x in words:
        key = (key << 64) | int(x)
    e = [0] * (k + 1)
    e[k] = key & 3
    for i in range(k):
        e[i] = (key >> (2 * (i + 1))) & 3
    return "".join(_BASES[c] for c in e)


def removed_tips(edges: list[str], max_len: int) -> set[str]:
    """Edges ((k+1)-mer strings) that tip removal takes out of the graph."""
    out_e: dict[str, list[str]] = defaultdict(list)
    in_e: dict[str, list[str]] = defaultdict(list)
    nodes = set()
    for x in edges:
        out_e[x[:-1]].append(x)
        in_e[x[1:]].append(x)
        nodes.add(x[:-1])
        nodes.add(x[1:])

    def indeg(v):
        return len(in_e.get(v, ()))

    def outdeg(v):
        return len(out_e.get(v, ()))

    gone: set[str] = set()
    for v0 in nodes:
        # forward tip from a node without incoming edges
        if indeg(v0) == 0:
            path, cur = [], v0
            while outdeg(cur) == 1 and len(path) < max_len:
                x = out_e[cur][0]
                path.append(x)
                cur = x[1:]
                if indeg(cur) >= 2 or outdeg(cur) == 0:
                    gone.update(path)
                    break
                if indeg(cur) != 1:
                    break
        # backward tip into a node without outgoing edges
        if outdeg(v0) == 0:
            path, cur = [], v0
            while indeg(cur) == 1 and len(path) < max_len:
                x = in_e[cur][0]
                path.append(x)
                cur = x[:-1]
                if outdeg(cur) >= 2 or indeg(cur) == 0:
                    gone.update(path)
                    break
                if outdeg(cur) != 1:
                    break
    return gone


def removed_mask(keys: np.ndarray, k: int, max_len: int) -> np.ndarray:
    """For sorted edge keys (rows of w words), a bool array marking the edges
    tip removal takes out."""
    keys = np.asarray(keys, dtype=np.uint64).reshape(len(keys), -1)
    edges = [key_to_edge(row, k) for row in keys]
    gone = removed_tips(edges, max_len)
    return np.array([x in gone for x in edges], dtype=bool)
