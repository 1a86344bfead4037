"""Navigation on the device (sdbg_index_build, sdbg_navigate) against the
explicit graph: for every row and every node, the node, forward target,
backward source, out- and in-degree and k-mer agree with the rows built
from the edge set by their definitions (real rows, one '$' row per vertex
with no outgoing edge, one dummy row per vertex with no incoming edge)."""

from __future__ import annotations

import json
import os

import numpy as np
import pytest

import brute
import oracle
from gpu_util import gpu_count, say
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu
NONE = np.uint64(0xFFFFFFFFFFFFFFFF)
RANK = {"$": 0, "A": 1, "C": 2, "G": 3, "T": 4}
HERE = os.path.dirname(os.path.abspath(__file__))


def _explicit_rows(edges: list[str], k: int):
    """(source, label, kind) of every row in row order; kind 0 real, 1 '$', 2 dummy."""
    P = {e[:k] for e in edges}
    Q = {e[1:] for e in edges}
    rows = [(e[:k], e[k], 0) for e in edges]
    rows += [(v, "$", 1) for v in Q - P]
    rows += [("$" + v[: k - 1], v[k - 1], 2) for v in P - Q]
    rows.sort(key=lambda r: tuple(RANK[ch] for ch in reversed(r[0])) + (RANK[r[1]],))
    return rows


def _check_nav(rs, k, d, mercy):
    e, keys, cnt = gpu_count(rs, k, d, mercy)
    g = sdbg.build(e)
    h = g.to_host()
    edges = [brute.key_to_edge(brute.words_to_key(row), k) for row in keys]
    rows = _explicit_rows(edges, k)
    m = len(rows)
    assert m == h.m
    # nodes: runs of rows with one source; id = index of the run's last row
    node_id = [0] * m
    last_of = {}
    for i in range(m - 1, -1, -1):
        if i == m - 1 or rows[i + 1][0] != rows[i][0]:
            last_of[rows[i][0]] = i
        node_id[i] = last_of[rows[i][0]]
    size = {}
    for u in node_id:
        size[u] = size.get(u, 0) + 1
    first_in = {}  # target k-mer -> first row entering it (real or dummy)
    indeg = {}
    for i, (src, lab, kind) in enumerate(rows):
        if lab == "$":
            continue
        tgt = src[1:] + lab
        first_in.setdefault(tgt, i)
        if kind == 0:
            indeg[tgt] = indeg.get(tgt, 0) + 1
    exp = {op: np.full(m, NONE, dtype=np.uint64) for op in range(1, 6)}
    lw = (2 * k + 63) // 64
    exp_label = np.full((m, lw), NONE, dtype=np.uint64)
    for i, (src, lab, kind) in enumerate(rows):
        u = node_id[i]
        exp[sdbg.NAV_NODE][i] = u
        if lab != "$":
            exp[sdbg.NAV_FORWARD][i] = last_of[src[1:] + lab]
        dummy = src.startswith("$")
        exp[sdbg.NAV_OUTDEG][i] = 0 if rows[u][1] == "$" else size[u]
        if not dummy:
            exp[sdbg.NAV_BACKWARD][i] = node_id[first_in[src]]
            exp[sdbg.NAV_INDEG][i] = indeg.get(src, 0)
            word = 0
            for j, ch in enumerate(src):
                word |= "ACGT".index(ch) << (2 * j)
            exp_label[i] = [(word >> (64 * q)) & 0xFFFFFFFFFFFFFFFF for q in range(lw)]
        else:
            exp[sdbg.NAV_INDEG][i] = 0
    import torch

    ix = sdbg.Index(g)
    q = torch.arange(m + 3, dtype=torch.int64, device="cuda")  # three rows past the end: all ones
    for op in range(1, 6):
        out = torch.zeros(m + 3, dtype=torch.int64, device="cuda")
        ix.navigate(op, q, out)
        got = out.cpu().numpy().view(np.uint64)
        assert (got[m:] == NONE).all()
        bad = np.flatnonzero(got[:m] != exp[op])
        assert bad.size == 0, f"op {op}: {bad.size} rows differ, first row {bad[0]}: {got[bad[0]]} vs {exp[op][bad[0]]}"
    out = torch.zeros((m + 3) * lw, dtype=torch.int64, device="cuda")
    ix.navigate(sdbg.NAV_LABEL, q, out)
    got = out.cpu().numpy().view(np.uint64).reshape(m + 3, lw)
    assert np.array_equal(got[:m], exp_label) and (got[m:] == NONE).all()
    ix.close()
    g.close()
    e.close()
    say(f"  navigation ok: {m} rows, k={k}")


with open(os.path.join(HERE, "golden", "toys.json")) as f:
    TOYS = json.load(f)["toys"]


@pytest.mark.parametrize("toy", TOYS, ids=[t["name"] for t in TOYS])
def test_navigation_toys(toy):
    _check_nav(synth.from_strings(toy["reads"], toy["k"], toy["d"], toy["mercy"]), toy["k"], toy["d"], toy["mercy"])


@pytest.mark.parametrize("k", [5, 21, 31, 32, 41, 63, 64, 81, 99, 127])
def test_navigation_random(k):
    rs = synth.random_small(150, 60, 250, 1500, 0.01, seed=300 + k, n_rate=0.005)
    _check_nav(rs, k, 2, True)


def test_navigation_tiny_workload():
    _check_nav(synth.tiny(scale=0.02), 21, 2, True)
