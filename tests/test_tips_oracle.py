"""Pins of the tip-removal oracle (oracle/tips.py) on hand-built graphs
whose tips are known by construction: a main path with a short branch
joining it or leaving it, a branch one edge too long, an isolated short
path, a bubble, and a branch that splits again (not a simple path)."""

from __future__ import annotations

import random

from oracle import tips

K = 7


def edges_of(*seqs: str) -> set[str]:
    out = set()
    for s in seqs:
        for i in range(len(s) - K):
            out.add(s[i : i + K + 1])
    return out


def rand_seq(n: int, rng: random.Random, first_not: str = "", last_not: str = "") -> str:
    """n random bases; the first is not first_not and the last not last_not
    (so that a branch meets the main path exactly where it is built to)."""
    while True:
        x = "".join(rng.choice("ACGT") for _ in range(n))
        if x[:1] != first_not and x[-1:] != last_not:
            return x


def main_path(rng, n=80):
    # a path whose k-mers are all distinct (so it is a simple path)
    while True:
        s = rand_seq(n, rng)
        kms = [s[i : i + K] for i in range(n - K + 1)]
        if len(set(kms)) == len(kms):
            return s


def test_branch_joining_is_removed():
    rng = random.Random(1)
    s = main_path(rng)
    p = 40  # far from both ends (more than max_len edges)
    branch = rand_seq(3, rng, last_not=s[p - 1]) + s[p : p + K]  # 3 new edges ending in s's node at p
    E = edges_of(s, branch)
    got = tips.removed_tips(sorted(E), max_len=10)
    assert got == edges_of(branch)


def test_branch_leaving_is_removed():
    rng = random.Random(2)
    s = main_path(rng)
    p = 35
    branch = s[p : p + K] + rand_seq(4, rng, first_not=s[p + K])  # leaves s's node at p, ends after 4 edges
    E = edges_of(s, branch)
    assert tips.removed_tips(sorted(E), max_len=10) == edges_of(branch)


def test_branch_longer_than_max_len_is_kept():
    rng = random.Random(3)
    s = main_path(rng)
    p = 40
    branch = rand_seq(11, rng, last_not=s[p - 1]) + s[p : p + K]  # 11 edges
    E = edges_of(s, branch)
    assert tips.removed_tips(sorted(E), max_len=10) == set()
    assert tips.removed_tips(sorted(E), max_len=11) == edges_of(branch)


def test_isolated_short_path():
    rng = random.Random(4)
    s = main_path(rng, n=K + 3)  # 3 edges, no branches
    E = edges_of(s)
    assert tips.removed_tips(sorted(E), max_len=3) == E
    assert tips.removed_tips(sorted(E), max_len=2) == set()


def test_bubble_is_not_a_tip():
    rng = random.Random(5)
    s = main_path(rng)
    p = 30
    # a second path from s's node at p to s's node at p + K + 4 (a bubble)
    alt = s[p : p + K] + rand_seq(4, rng, first_not=s[p + K], last_not=s[p + K + 3]) + s[p + K + 4 : p + 2 * K + 4]
    E = edges_of(s, alt)
    assert tips.removed_tips(sorted(E), max_len=10) == set()


def test_splitting_branch_is_not_a_simple_tip():
    rng = random.Random(6)
    s = main_path(rng)
    p = 40
    stem = rand_seq(2, rng, last_not=s[p - 1]) + s[p : p + K]  # joins s after 2 edges ...
    fork = stem[:K] + rand_seq(2, rng, first_not=stem[K])  # ... but its first node also leads elsewhere
    E = edges_of(s, stem, fork)
    got = tips.removed_tips(sorted(E), max_len=10)
    # the stem's first node has out-degree 2, so no forward tip starts there;
    # the fork ends in a dead end, so its backward walk stops at that node
    # (out-degree 2) and the fork is a backward tip
    assert got == edges_of(fork)


def test_keys_round_trip():
    rng = random.Random(7)
    for k in (2, 21, 31, 32, 63, 99):
        e = rand_seq(k + 1, rng)
        key = int(e[k] == "A" and 0 or "ACGT".index(e[k]))
        for i in range(k):
            key += "ACGT".index(e[i]) << (2 * (i + 1))
        w = (2 * (k + 1) + 63) // 64
        words = [(key >> (64 * (w - 1 - j))) & (2**64 - 1) for j in range(w)]
        assert tips.key_to_edge(words, k) == e
