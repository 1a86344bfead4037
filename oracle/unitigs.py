"""TEST INFRASTRUCTURE ONLY: unitigs of the explicit de Bruijn graph.

Section 2 (fourth paragraph, and the workflow of its Fig. 1) passes contigs
from one k to the next; the paper gives no construction, so this follows the
reading fixed for the device path.  On the graph of the valid edges (those
of E that cleaning has not removed), with degrees counted over valid edges:

* a unitig is a maximal path in which every node between two consecutive
  edges has in-degree 1 and out-degree 1;
* every valid edge lies on exactly one unitig: a unitig starts at an edge
  whose source node is not (in-degree 1, out-degree 1) and follows the
  unique outgoing edge while the node reached is (in 1, out 1); a cycle whose
  nodes are all (in 1, out 1) is one unitig that starts at its first edge in
  the edge order;
* a unitig of L edges spells the k-mer of its first source node followed by
  the last base of each edge (k + L bases; for a cycle the last k bases
  repeat the first k); its multiplicity is the sum of its edges' counts.

Unitigs are listed in the edge order of their first edges.  Plain Python
over strings: nodes are k-mers, edge (k+1)-mer x goes from x[:-1] to x[1:].
"""

from __future__ import annotations

from collections import defaultdict


def unitigs(edges: list[str], counts, valid) -> list[tuple[int, int, int, str]]:
    """edges: (k+1)-mer strings in the edge order; counts and valid: one per
    edge.  Returns (index of the first edge, edges, multiplicity, sequence)
    per unitig, ascending in the first index."""
    idx = {x: i for i, x in enumerate(edges)}
    live = [x for x, ok in zip(edges, valid) if ok]
    out_e: dict[str, list[str]] = defaultdict(list)
    in_e: dict[str, list[str]] = defaultdict(list)
    for x in live:
        out_e[x[:-1]].append(x)
        in_e[x[1:]].append(x)

    def one_in_one_out(v: str) -> bool:
        return len(in_e.get(v, ())) == 1 and len(out_e.get(v, ())) == 1

    seen: set[str] = set()
    res = []

    def walk(first: str):
        path = [first]
        seen.add(first)
        v = first[1:]
        while one_in_one_out(v):
            nxt = out_e[v][0]
            if nxt in seen:  # back at the start of a cycle
                break
            path.append(nxt)
            seen.add(nxt)
            v = nxt[1:]
        seq = path[0] + "".join(x[-1] for x in path[1:])
        res.append((idx[first], len(path), sum(int(counts[idx[x]]) for x in path), seq))

    for x in live:  # starts: source node not (in 1, out 1)
        if not one_in_one_out(x[:-1]):
            walk(x)
    for x in sorted(live, key=idx.__getitem__):  # what is left lies on cycles
        if x not in seen:
            walk(x)
    res.sort()
    return res
