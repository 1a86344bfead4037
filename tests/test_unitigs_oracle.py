"""Pins of the unitig oracle (oracle/unitigs.py): hand-built graphs whose
unitigs are known by construction (a simple path, a branch joining or
leaving it, a bubble, a cycle, a self-loop, removed edges), and on random
graphs the defining properties checked by code of its own: the unitigs
partition the valid edges, consecutive edges meet at a node of in- and
out-degree 1, no unitig can be extended, sequences spell their edges and
multiplicities add up their counts."""

from __future__ import annotations

import random
from collections import Counter

import pytest

import brute
from oracle import unitigs as U
from test_tips_oracle import K, edges_of, main_path, rand_seq


def run(E, valid_pred=lambda x: True, counts=None):
    edges = sorted(E, key=brute.edge_key)
    cnt = counts or {x: 1 + (brute.edge_key(x) % 5) for x in edges}
    res = U.unitigs(edges, [cnt[x] for x in edges], [valid_pred(x) for x in edges])
    return edges, cnt, res


def seqs(res):
    return sorted(r[3] for r in res)


def test_simple_path_is_one_unitig():
    s = main_path(random.Random(1))
    edges, cnt, res = run(edges_of(s))
    assert len(res) == 1
    first, n, mult, seq = res[0]
    assert seq == s and n == len(s) - K and mult == sum(cnt.values())
    assert edges[first] == s[: K + 1]


def test_branch_joining_splits_the_path():
    rng = random.Random(2)
    s = main_path(rng)
    p = 40
    branch = rand_seq(3, rng, last_not=s[p - 1]) + s[p : p + K]
    _, _, res = run(edges_of(s, branch))
    # node s[p:p+K] has in-degree 2
    assert seqs(res) == sorted([s[: p + K], s[p:], branch])


def test_branch_leaving_splits_the_path():
    rng = random.Random(3)
    s = main_path(rng)
    p = 35
    branch = s[p : p + K] + rand_seq(4, rng, first_not=s[p + K])
    _, _, res = run(edges_of(s, branch))
    assert seqs(res) == sorted([s[: p + K], s[p:], branch])


def test_bubble_gives_four_unitigs():
    rng = random.Random(4)
    s = main_path(rng)
    p = 30
    q = p + K + 4
    alt = s[p : p + K] + rand_seq(4, rng, first_not=s[p + K], last_not=s[q - 1]) + s[q : q + K]
    _, _, res = run(edges_of(s, alt))
    assert seqs(res) == sorted([s[: p + K], s[p : q + K], alt, s[q:]])


def test_cycle_starts_at_its_first_edge_in_edge_order():
    rng = random.Random(5)
    while True:  # a circular sequence whose k-mers (cyclically) are distinct
        c = rand_seq(30, rng)
        c2 = c + c[:K]
        kms = [c2[i : i + K] for i in range(len(c))]
        if len(set(kms)) == len(kms):
            break
    E = {c2[i : i + K + 1] for i in range(len(c))}
    edges, cnt, res = run(E)
    assert len(res) == 1
    first, n, mult, seq = res[0]
    assert first == 0 and n == len(c) and mult == sum(cnt.values())
    j = c2.index(edges[0])  # the cycle read from its smallest edge
    rot = c[j:] + c[:j]
    assert seq == rot + rot[:K]


def test_self_loop():
    x = "A" * (K + 1)
    _, _, res = run({x}, counts={x: 7})
    assert res == [(0, 1, 7, x)]


def test_removed_edges_are_not_on_unitigs():
    rng = random.Random(6)
    s = main_path(rng)
    p = 40
    branch = rand_seq(3, rng, last_not=s[p - 1]) + s[p : p + K]
    gone = edges_of(branch)
    _, _, res = run(edges_of(s, branch), valid_pred=lambda x: x not in gone)
    assert seqs(res) == [s]  # node p is back to in-degree 1
    # removing an edge in the middle of the path cuts it in two
    mid = s[50 : 51 + K]
    _, _, res = run(edges_of(s), valid_pred=lambda x: x != mid)
    assert seqs(res) == sorted([s[: 50 + K], s[51:]])


def _check_properties(edges, cnt, valid, res):
    live = [x for x, ok in zip(edges, valid) if ok]
    indeg, outdeg = Counter(), Counter()
    for x in live:
        outdeg[x[:-1]] += 1
        indeg[x[1:]] += 1
    mid = lambda v: indeg[v] == 1 and outdeg[v] == 1  # noqa: E731
    covered = []
    assert [r[0] for r in res] == sorted(r[0] for r in res)
    for first, n, mult, seq in res:
        path = [seq[i : i + K + 1] for i in range(n)]
        assert len(seq) == n + K and path[0] == edges[first]
        covered += path
        assert mult == sum(cnt[x] for x in path)
        for a, b in zip(path, path[1:]):  # joined through a node of in 1 / out 1
            assert a[1:] == b[:-1] and mid(a[1:])
        cyc = seq[:K] == seq[-K:] and mid(seq[:K])
        if cyc:  # a cycle starts at its smallest edge
            assert first == min(edges.index(x) for x in path)
        else:  # maximal at both ends
            assert not mid(path[0][:-1]) and not mid(path[-1][1:])
    assert sorted(covered) == sorted(live)  # every valid edge exactly once


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_properties(seed):
    rng = random.Random(100 + seed)
    g = rand_seq(300, rng)
    if seed % 2:  # a repeat, so that nodes of in/out-degree 2 occur
        g = g[:150] + g[20:60] + g[150:]
    reads = []
    for _ in range(120):
        i = rng.randrange(0, len(g) - 30)
        r = list(g[i : i + 30])
        if rng.random() < 0.3:
            r[rng.randrange(30)] = rng.choice("ACGT")
        reads.append("".join(r))
    E = set()
    for r in reads:
        E |= edges_of(r)
    edges = sorted(E, key=brute.edge_key)
    cnt = {x: rng.randint(1, 9) for x in edges}
    valid = [rng.random() < 0.9 for _ in edges]
    res = U.unitigs(edges, [cnt[x] for x in edges], valid)
    _check_properties(edges, cnt, valid, res)
