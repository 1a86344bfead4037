"""Independent brute-force reference pieces used to pin the oracle.

Written directly from the definitions, with Python strings and sets, sharing
no code with the oracle (C++) or the device library:

* ``edge_key`` -- the colex sort key of a (k+1)-mer (Section 2, second
  paragraph): digits e[k-1], ..., e[0], then the label e[k], read as one
  base-4 number via ``int(.., 4)``;
* ``brute_edges`` -- both-strand counting, solid filter and the mercy rule
  (Section 2, third paragraph) over all pairs of solid positions of a read;
* ``decode_sdbg`` -- reads a graph back out of the SdBG arrays by navigation
  alone (the O(1) traversal of Section 2, first paragraph): each node's k-mer
  is recovered by walking incoming edges backwards through F, the minus flags
  and the last bits, falling back to the 2kt-bit tip vector for dummy
  nodes.  It never looks at how the arrays were built.
"""

from __future__ import annotations

import math

import numpy as np

BASES = "ACGT"
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def revcomp(s: str) -> str:
    return "".join(COMP[c] for c in reversed(s))


def segments(reads: list[bytes]) -> list[str]:
    out = []
    for r in reads:
        cur = []
        for ch in r.decode("latin-1"):
            u = ch.upper()
            if u in COMP:
                cur.append(u)
            else:
                if cur:
                    out.append("".join(cur))
                cur = []
        if cur:
            out.append("".join(cur))
    return out


def edge_key(e: str) -> int:
    k = len(e) - 1
    digits = e[k - 1 :: -1] + e[k]
    return int("".join(str(BASES.index(c)) for c in digits), 4)


def key_to_words(key: int, k: int) -> list[int]:
    w = math.ceil(2 * (k + 1) / 64)
    return [(key >> (64 * (w - 1 - i))) & ((1 << 64) - 1) for i in range(w)]


def words_to_key(words) -> int:
    v = 0
    for x in words:
        v = (v << 64) | int(x)
    return v


def key_to_edge(key: int, k: int) -> str:
    digits = []
    for _ in range(k + 1):
        digits.append(BASES[key & 3])
        key >>= 2
    # digits[0] = label e[k], digits[1] = e[0], ..., digits[k] = e[k-1]
    return "".join(digits[1:]) + digits[0]


def brute_counts(reads: list[bytes], k: int) -> dict[str, int]:
    cnt: dict[str, int] = {}
    for s in segments(reads):
        for i in range(len(s) - k):
            x = s[i : i + k + 1]
            for y in (x, revcomp(x)):
                cnt[y] = cnt.get(y, 0) + 1
    return cnt


def brute_edges(reads: list[bytes], k: int, d: int, mercy: bool):
    """Returns (dict edge -> count for E, set of mercy edges)."""
    cnt = brute_counts(reads, k)
    solid = {x for x, c in cnt.items() if c >= d}
    mercy_set: set[str] = set()
    if mercy:
        for s in segments(reads):
            wins = [s[i : i + k + 1] for i in range(len(s) - k)]
            for p in range(len(wins)):
                for q in range(p + 2, len(wins)):
                    x, y = wins[p], wins[q]
                    if x not in solid or y not in solid:
                        continue
                    if any(wins[i] in solid for i in range(p + 1, q)):
                        continue
                    # x has no outgoing solid edge, y has no incoming one
                    if any(x[1:] + c in solid for c in BASES):
                        continue
                    if any(c + y[:-1] in solid for c in BASES):
                        continue
                    for i in range(p + 1, q):
                        mercy_set.add(wins[i])
                        mercy_set.add(revcomp(wins[i]))
    E = {x: cnt[x] for x in solid | mercy_set}
    return E, mercy_set


def expected_graph(E: dict[str, int], k: int):
    """Explicit graph the SdBG must encode: node -> {label: mult}."""
    P = {e[:k] for e in E}
    Q = {e[1:] for e in E}
    nodes: dict[str, dict[str, int]] = {}
    for e, c in E.items():
        nodes.setdefault(e[:k], {})[e[k]] = c
    for v in Q - P:
        nodes.setdefault(v, {})["$"] = 0
    for v in P - Q:
        nodes.setdefault("$" + v[: k - 1], {})[v[k - 1]] = 0
    return nodes, Q - P, P - Q


def _bit(words: np.ndarray, i: int) -> int:
    return int((int(words[i // 64]) >> (i % 64)) & 1)


def decode_sdbg(W, last, valid, tip, mult, F, tip_seq, m: int, k: int):
    """Navigation-only decoder.  Returns (nodes, edges, checks) where nodes maps
    each node's string to {label: mult}, edges maps real edges to mult.
    Raises AssertionError on any structural inconsistency."""
    W = np.asarray(W)
    lab = [int(x) & 7 for x in W]
    minus = [(int(x) >> 3) & 1 for x in W]
    is_last = [_bit(last, i) for i in range(m)]
    is_tip = [_bit(tip, i) for i in range(m)]
    is_valid = [_bit(valid, i) for i in range(m)]
    assert m == 0 or is_last[m - 1] == 1
    assert int(F[5]) == m and int(F[0]) == 0
    assert all(int(F[c]) <= int(F[c + 1]) for c in range(5))
    # nodes = maximal runs closed by a last bit
    node_of_row, node_first = [], []
    n = 0
    for i in range(m):
        if i == 0 or is_last[i - 1]:
            node_first.append(i)
        node_of_row.append(len(node_first) - 1)
    n_nodes = len(node_first)
    node_rows = [[] for _ in range(n_nodes)]
    for i in range(m):
        node_rows[node_of_row[i]].append(i)
    # block (last symbol of the node, 1..4) from F
    def block(i):
        for c in range(1, 5):
            if int(F[c]) <= i < int(F[c + 1]):
                return c
        raise AssertionError("row outside F blocks")
    node_block = [block(node_first[v]) for v in range(n_nodes)]
    for v in range(n_nodes):
        assert all(block(i) == node_block[v] for i in node_rows[v])
    # a dummy node owns only tip rows, a real node none
    node_is_tip = []
    for v in range(n_nodes):
        ts = {is_tip[i] for i in node_rows[v]}
        assert len(ts) == 1, "node mixes tip and non-tip rows"
        node_is_tip.append(ts.pop() == 1)
    # tip k-mers in row order
    tip_rank = {}
    r = 0
    for i in range(m):
        if is_tip[i]:
            tip_rank[i] = r
            r += 1
    t = r
    assert len(tip_seq) == (2 * k * t + 63) // 64

    def tip_kmer(i):
        rr = tip_rank[i]
        return "".join(BASES[(int(tip_seq[(2 * (k * rr + j)) // 64]) >> ((2 * (k * rr + j)) % 64)) & 3] for j in range(k))

    # rank of unflagged c-rows <-> non-tip nodes of block c
    unflagged = {c: [i for i in range(m) if lab[i] == c and not minus[i]] for c in range(1, 5)}
    nontip_nodes = {c: [v for v in range(n_nodes) if node_block[v] == c and not node_is_tip[v]] for c in range(1, 5)}
    for c in range(1, 5):
        assert len(unflagged[c]) == len(nontip_nodes[c]), "I10: unflagged c-rows != non-tip nodes in block c"
    incoming = {}  # non-tip node -> row of its unflagged incoming edge
    for c in range(1, 5):
        for row, v in zip(unflagged[c], nontip_nodes[c]):
            incoming[v] = row

    def forward(i):
        c = lab[i]
        if c == 0:
            return None
        j = i
        if minus[i]:
            j = max(x for x in unflagged[c] if x < i)
        return nontip_nodes[c][unflagged[c].index(j)]

    memo: dict[int, str] = {}

    def node_str(v):
        if v in memo:
            return memo[v]
        syms = []
        u = v
        while len(syms) < k:
            if node_is_tip[u]:
                vv = tip_kmer(node_rows[u][0])
                # '$' + v[0..k-2]; the remaining (older) symbols come from it
                full = "$" + vv[: k - 1]
                need = k - len(syms)
                s = full[-need:] + "".join(reversed(syms)) if need > 0 else "".join(reversed(syms))
                memo[v] = s
                return s
            syms.append(BASES[node_block[u] - 1])
            u = node_of_row[incoming[u]]
        s = "".join(reversed(syms))
        memo[v] = s
        return s

    nodes: dict[str, dict[str, int]] = {}
    edges: dict[str, int] = {}
    for v in range(n_nodes):
        s = node_str(v)
        assert s not in nodes, f"duplicate node {s}"
        d = {}
        for i in node_rows[v]:
            L = "$" if lab[i] == 0 else BASES[lab[i] - 1]
            assert L not in d, "two rows of one node share a label"
            d[L] = int(mult[i]) if is_valid[i] else 0
            if is_tip[i]:
                assert tip_kmer(i)[: k - 1] == s[1:] and s[0] == "$"
                assert tip_kmer(i)[k - 1] == L
                assert not is_valid[i] and not minus[i]
            if lab[i] == 0:
                assert not is_valid[i] and not minus[i]
        nodes[s] = d
    for i in range(m):
        s = node_str(node_of_row[i])
        if lab[i] == 0:
            continue
        L = BASES[lab[i] - 1]
        tgt = node_str(forward(i))
        assert tgt == s[1:] + L, f"forward({i}) reached {tgt}, expected {s[1:] + L}"
        if is_valid[i]:
            edges[s + L] = int(mult[i])
    # rows in colex order of source, then label ($ < A < C < G < T)
    rank = {"$": 0, "A": 1, "C": 2, "G": 3, "T": 4}
    order = []
    for i in range(m):
        s = node_str(node_of_row[i])
        L = "$" if lab[i] == 0 else BASES[lab[i] - 1]
        order.append(tuple(rank[ch] for ch in reversed(s)) + (rank[L],))
    assert all(order[i] < order[i + 1] for i in range(m - 1)), "rows not in colex order"
    return nodes, edges
