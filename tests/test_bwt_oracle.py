"""Pins of the read-set BWT oracle (oracle/bwt.py): a worked example, the
textbook BWT of one string (last column of its sorted rotations) for random
single reads, two identical reads (ties by read index), and for random read
sets (with duplicates, short and empty reads) the inversion by LF mapping,
written here on its own, which must give back every read."""

from __future__ import annotations

import random

from oracle import bwt


def test_worked_example():
    order, b = bwt.read_bwt(["ACG"])
    assert order == [(0, 3), (0, 0), (0, 1), (0, 2)]  # $, ACG$, CG$, G$
    assert b == "G$AC"
    order, b = bwt.read_bwt(["AC", "AC"])
    assert order == [(0, 2), (1, 2), (0, 0), (1, 0), (0, 1), (1, 1)]
    assert b == "CC$$AA"


def _rotation_bwt(s: str) -> str:
    t = s + "!"  # '!' sorts before the bases, as the end marker
    rots = sorted(t[i:] + t[:i] for i in range(len(t)))
    return "".join(r[-1] for r in rots).replace("!", "$")


def test_single_read_is_the_textbook_bwt():
    rng = random.Random(1)
    for n in (1, 2, 5, 17, 60):
        for _ in range(20):
            s = "".join(rng.choice("ACGT") for _ in range(n))
            assert bwt.read_bwt([s])[1] == _rotation_bwt(s)


def _invert(b: str, n_reads: int) -> list[str]:
    """Reads back from a multi-string BWT: rows 0..n-1 are the end markers in
    read order; LF mapping walks each read backwards to its '$'."""
    order = "$ACGT"
    C, tot = {}, 0
    for c in order:
        C[c] = tot
        tot += b.count(c)
    occ = {c: [0] * (len(b) + 1) for c in order}
    for i, ch in enumerate(b):
        for c in order:
            occ[c][i + 1] = occ[c][i] + (ch == c)
    reads = []
    for r in range(n_reads):
        row, out = r, []
        while b[row] != "$":
            c = b[row]
            out.append(c)
            row = C[c] + occ[c][row]
        reads.append("".join(reversed(out)))
    return reads


def test_inversion_gives_back_the_reads():
    rng = random.Random(2)
    for trial in range(30):
        reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 30))) for _ in range(rng.randint(1, 25))]
        if trial % 3 == 0:  # duplicates and shared prefixes
            reads += reads[: len(reads) // 2] + [x[:5] for x in reads[:3]]
        order, b = bwt.read_bwt(reads)
        assert len(b) == sum(len(x) + 1 for x in reads) == len(order)
        assert sorted(order) == sorted((r, j) for r, x in enumerate(reads) for j in range(len(x) + 1))
        assert _invert(b, len(reads)) == reads
