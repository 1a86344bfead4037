"""TEST INFRASTRUCTURE ONLY: the sorted suffixes of a read set and their BWT.

Section 2 (second paragraph) says MEGAHIT adapts CX1's construction, whose
core is sorting the suffixes of all reads into a Burrows-Wheeler transform
of the read set.  The paper gives no details; the reading fixed for the
device path is the usual multi-string BWT: each read r is followed by its
own end marker $_r, smaller than every base, with $_r < $_s when r < s.
Every read of length L has L + 1 suffixes (the last is $_r alone); they are
sorted by that order, and the BWT holds, for each suffix in sorted order,
the character before it in its read ('$' for a suffix that starts its
read).

Plain Python: the suffixes are compared as lists of base codes, where a
list that is a proper prefix of another sorts first (the end marker), and
equal lists by read index.
"""

from __future__ import annotations

_CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def suffix_order(reads: list[str]) -> list[tuple[int, int]]:
    """(read, offset) of every suffix in sorted order."""
    sufs = []
    for r, s in enumerate(reads):
        codes = [_CODE[c] for c in s.upper()]
        for j in range(len(codes) + 1):
            sufs.append((codes[j:], r, j))
    sufs.sort(key=lambda x: (x[0], x[1]))
    return [(r, j) for _, r, j in sufs]


def read_bwt(reads: list[str]) -> tuple[list[tuple[int, int]], str]:
    """The sorted suffixes and the BWT string ('$', 'A', 'C', 'G', 'T')."""
    order = suffix_order(reads)
    ups = [s.upper() for s in reads]
    return order, "".join("$" if j == 0 else ups[r][j - 1] for r, j in order)
