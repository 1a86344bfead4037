"""Host replay (CPU) of the schedule the device's read-set BWT follows
(paper_1409_7208_amd/csrc/bwt.hip): first keys of 21 characters (3 bits
each, the end marker and all after it 0), groups named by the place of their
first suffix, each round re-sorting only the suffixes of shared groups by
(group of the first h characters, group of the next h) or, when the end
marker lies within the first h, (group, read index), and splitting groups in
place.  Plain Python sorts stand in for the radix passes; the order must be
the oracle's (oracle/bwt.py) on random read sets, duplicates, homopolymers
(many rounds) and periodic reads."""

from __future__ import annotations

import random

import pytest

from oracle import bwt as ob

FIRST = 21


def replay(reads: list[str]) -> list[tuple[int, int]]:
    n = len(reads)
    off = [0]
    for x in reads:
        off.append(off[-1] + len(x))
    N = off[-1] + n
    rid = [0] * N
    for r in range(n):
        for p in range(off[r] + r, off[r + 1] + r + 1):
            rid[p] = r
    code = {"A": 1, "C": 2, "G": 3, "T": 4}
    seq = "".join(reads)

    def first_key(p):
        r = rid[p]
        j, L = p - (off[r] + r), off[r + 1] - off[r]
        k = 0
        for t in range(FIRST):
            k = (k << 3) | (code[seq[off[r] + j + t]] if j + t < L else 0)
        return k

    todo, place = list(range(N)), None  # suffixes to order and their places (None: 0..N-1)
    keys = {p: first_key(p) for p in todo}
    grp, sa, h = [0] * N, [0] * N, FIRST
    while True:
        srt = sorted(todo, key=lambda p: keys[p])  # stable, as the radix passes
        pos = (lambda i: i) if place is None else place.__getitem__
        heads = [i for i in range(len(srt)) if i == 0 or keys[srt[i]] != keys[srt[i - 1]]] + [len(srt)]
        nxt, nplace = [], []
        for a, b in zip(heads, heads[1:]):
            for i in range(a, b):
                p = srt[i]
                grp[p] = pos(a)
                sa[pos(i)] = p
                if b - a > 1:
                    nxt.append(p)
                    nplace.append(pos(i))
        if not nxt:
            break
        todo, place = nxt, nplace
        keys = {}
        for p in todo:
            r = rid[p]
            end = off[r + 1] + r
            second = r if end - p + 1 <= h else n + grp[p + h]
            keys[p] = grp[p] * (N + n) + second
        h *= 2
    return [(rid[p], p - (off[rid[p]] + rid[p])) for p in sa]


@pytest.mark.parametrize("seed", range(8))
def test_replay_equals_oracle(seed):
    rng = random.Random(900 + seed)
    for trial in range(25):
        reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 70))) for _ in range(rng.randint(1, 12))]
        if trial % 4 == 0:
            reads += reads[:3] + [x[:30] for x in reads[:2]]
        if trial % 5 == 0:
            reads = ["A" * rng.randint(0, 60) for _ in range(5)]
        if trial % 7 == 0:
            reads = ["ACGTTGCA"[: rng.randint(1, 8)] * rng.randint(1, 9) for _ in range(6)]
        assert replay(reads) == ob.suffix_order(reads), reads
