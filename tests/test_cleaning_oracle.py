"""Pins of the bubble and low-local-coverage oracle (oracle/cleaning.py) on
hand-built graphs whose outcome is known by construction: a two-branch
bubble with a weak branch, a tie, a bubble longer than max_len, a three-way
bubble, a weakly covered branch next to a well covered path (removed), a
well covered one (kept), an isolated weak path (no neighbours: kept), and
the neighbour mean taken over both ends."""

from __future__ import annotations

import random

import brute
from oracle import cleaning
from test_tips_oracle import K, edges_of, main_path, rand_seq


def _run(fn, E, cnt, *args):
    edges = sorted(E, key=brute.edge_key)
    return fn(edges, [cnt[x] for x in edges], [True] * len(edges), K, *args)


def _bubble(rng, s, p=30, n_alt=4):
    q = p + K + n_alt
    return s[p : p + K] + rand_seq(n_alt, rng, first_not=s[p + K], last_not=s[q - 1]) + s[q : q + K]


def test_weak_branch_of_a_bubble_is_removed():
    rng = random.Random(1)
    s = main_path(rng)
    alt = _bubble(rng, s)
    cnt = {x: 10 for x in edges_of(s)} | {x: 2 for x in edges_of(alt)}
    assert _run(cleaning.bubbles, cnt.keys(), cnt, 20) == edges_of(alt)
    # the stronger branch stays whichever it is
    cnt2 = {x: 2 for x in edges_of(s)} | {x: 10 for x in edges_of(alt)}
    p, q = 30, 30 + K + 4
    assert _run(cleaning.bubbles, cnt2.keys(), cnt2, 20) == edges_of(s[p : q + K])


def test_tie_keeps_the_branch_with_the_smaller_first_edge():
    rng = random.Random(2)
    s = main_path(rng)
    alt = _bubble(rng, s)
    cnt = {x: 5 for x in edges_of(s, alt)}
    p, q = 30, 30 + K + 4
    main_seg = s[p : q + K]
    first = lambda seq: brute.edge_key(seq[: K + 1])  # noqa: E731
    loser = alt if first(main_seg) < first(alt) else main_seg
    assert _run(cleaning.bubbles, cnt.keys(), cnt, 20) == edges_of(loser)


def test_bubble_longer_than_max_len_is_kept():
    rng = random.Random(3)
    s = main_path(rng)
    alt = _bubble(rng, s)
    cnt = {x: 10 for x in edges_of(s)} | {x: 2 for x in edges_of(alt)}
    assert _run(cleaning.bubbles, cnt.keys(), cnt, K + 3) == set()  # branches have K + 4 edges
    assert _run(cleaning.bubbles, cnt.keys(), cnt, K + 4) == edges_of(alt)


def test_three_way_bubble_keeps_one():
    rng = random.Random(4)
    s = main_path(rng)
    a1 = _bubble(rng, s)
    while True:
        a2 = _bubble(rng, s)
        if not (edges_of(a2) & edges_of(a1)):
            break
    cnt = {x: 3 for x in edges_of(s)} | {x: 9 for x in edges_of(a1)} | {x: 4 for x in edges_of(a2)}
    p, q = 30, 30 + K + 4
    assert _run(cleaning.bubbles, cnt.keys(), cnt, 20) == edges_of(s[p : q + K], a2)


def test_weak_branch_next_to_a_covered_path_is_removed():
    rng = random.Random(5)
    s = main_path(rng)
    branch = rand_seq(3, rng, last_not=s[39]) + s[40 : 40 + K]  # joins s at node 40
    cnt = {x: 20 for x in edges_of(s)} | {x: 1 for x in edges_of(branch)}
    # neighbours at the branch's end: s's edges into and out of node 40 (20 each)
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 200) == edges_of(branch)
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 0) == set()
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 2, 200) == set()  # 3 edges > max_len
    # mean 1 against neighbours' mean 20: removed iff ratio > 1/20
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 50) == set()
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 51) == edges_of(branch)


def test_covered_branch_is_kept():
    rng = random.Random(6)
    s = main_path(rng)
    branch = s[35 : 35 + K] + rand_seq(4, rng, first_not=s[35 + K])
    cnt = {x: 20 for x in edges_of(s)} | {x: 15 for x in edges_of(branch)}
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 200) == set()


def test_isolated_weak_path_has_no_neighbours():
    rng = random.Random(7)
    s = main_path(rng, n=K + 4)
    cnt = {x: 1 for x in edges_of(s)}
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 10, 900) == set()


def test_neighbours_of_both_ends_count():
    rng = random.Random(8)
    s = main_path(rng)
    alt = _bubble(rng, s)  # starts at node 30, ends at node 30 + K + 4
    cnt = {x: 10 for x in edges_of(s)} | {x: 1 for x in edges_of(alt)}
    p, q = 30, 30 + K + 4
    # alt's neighbours: s's edges into p, out of p, into q, out of q (10 each);
    # the main segment between p and q is a unitig too, with alt's edges as
    # its neighbours at both ends (mean (10 + 1 + 1 + 10) / 4 = 5.5)
    assert _run(cleaning.low_coverage, cnt.keys(), cnt, 20, 100) == set()  # 1 is not below 0.1 * 10
    got = _run(cleaning.low_coverage, cnt.keys(), cnt, 20, 150)
    assert got == edges_of(alt)  # 1 < 0.15 * 10; the segment's 10 >= 0.15 * 5.5
