"""The identity the device's tip removal relies on, checked on the oracle's
definitions (CPU): the edges tip removal takes out (oracle/tips.py, walks
from the nodes without incoming or outgoing edges) are exactly the edges of
the unitigs of the graph as built (oracle/unitigs.py, every edge valid) of
at most max_len edges that are not cycles and whose end nodes have a tip's
degrees -- start without incoming edges, one outgoing, and an end that
joins the graph (in-degree >= 2) or stops (out-degree 0); or the mirror
image.  Random graphs with repeats, errors and short isolated pieces, and
every max_len from 1 to past the longest unitig."""

from __future__ import annotations

import random
from collections import Counter

import pytest

import brute
from oracle import tips
from oracle import unitigs as U


def _tips_from_unitigs(edges: list[str], k: int, max_len: int) -> set[str]:
    indeg, outdeg = Counter(), Counter()
    for x in edges:
        outdeg[x[:-1]] += 1
        indeg[x[1:]] += 1
    gone = set()
    for _, n, _, seq in U.unitigs(edges, [1] * len(edges), [True] * len(edges)):
        if n > max_len:
            continue
        s, t = seq[:k], seq[-k:]
        if indeg[s] == 1 and outdeg[s] == 1:  # a cycle
            continue
        fwd = indeg[s] == 0 and outdeg[s] == 1 and (indeg[t] >= 2 or outdeg[t] == 0)
        bwd = outdeg[t] == 0 and indeg[t] == 1 and (outdeg[s] >= 2 or indeg[s] == 0)
        if fwd or bwd:
            gone.update(seq[i : i + k + 1] for i in range(n))
    return gone


@pytest.mark.parametrize("seed", range(12))
def test_tips_are_unitigs_with_tip_ends(seed):
    rng = random.Random(500 + seed)
    k = rng.choice([5, 7, 9])
    g = "".join(rng.choice("ACGT") for _ in range(rng.randint(80, 400)))
    if seed % 3 == 0:  # repeats: nodes of in- or out-degree 2 inside the genome
        g = g[:60] + g[10:40] + g[60:] + g[25:55]
    reads = []
    for _ in range(rng.randint(20, 120)):
        i = rng.randrange(0, max(1, len(g) - 12))
        r = list(g[i : i + rng.randint(k + 1, 40)])
        if rng.random() < 0.4:  # an error: a bubble or a tip
            r[rng.randrange(len(r))] = rng.choice("ACGT")
        reads.append("".join(r))
    reads += ["".join(rng.choice("ACGT") for _ in range(rng.randint(k + 1, k + 6))) for _ in range(3)]  # islands
    E = set()
    for r in reads:
        E |= {r[i : i + k + 1] for i in range(len(r) - k)}
    edges = sorted(E, key=brute.edge_key)
    longest = max(n for _, n, _, _ in U.unitigs(edges, [1] * len(edges), [True] * len(edges)))
    for max_len in range(1, longest + 2):
        assert tips.removed_tips(edges, max_len) == _tips_from_unitigs(edges, k, max_len), max_len
