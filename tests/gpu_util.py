"""Helpers for the device tests: run the HIP path through the C ABI on
seeded inputs and compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np

from paper_1409_7208_amd import sdbg


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(rs):
    import torch

    seq = torch.from_numpy(np.ascontiguousarray(rs.seq)).to("cuda")
    off = torch.from_numpy(np.ascontiguousarray(rs.offsets).view(np.int64)).to("cuda")
    return seq, off


def gpu_count(rs, k, d, mercy, prefix_len=8, mem_budget=0, device_input=True):
    if device_input:
        seq, off = to_device(rs)
    else:
        seq, off = rs.seq, rs.offsets
    e = sdbg.count_solid(seq, off, k, d, mercy, prefix_len=prefix_len, mem_budget=mem_budget)
    keys, cnt = e.to_host()
    return e, keys, cnt


def gpu_graph(e):
    g = sdbg.build(e)
    h = g.to_host()
    g.close()
    return h


def assert_graph_equal(h, og):
    assert h.m == og.m and h.t == og.t
    assert np.array_equal(h.W, og.W)
    assert np.array_equal(h.last, og.last)
    assert np.array_equal(h.valid, og.valid)
    assert np.array_equal(h.tip, og.tip)
    assert np.array_equal(h.mult, og.mult)
    assert np.array_equal(h.F, og.F)
    assert np.array_equal(h.tip_seq, og.tip_seq)


def popcount(words: np.ndarray) -> int:
    w = np.asarray(words, dtype=np.uint64)
    return int(np.unpackbits(w.view(np.uint8)).sum())


def bits(words: np.ndarray, m: int) -> np.ndarray:
    w = np.asarray(words, dtype=np.uint64)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:m].astype(bool)


def revcomp_keys_w1(keys: np.ndarray, k: int) -> np.ndarray:
    """Keys of the reverse complements, for one-word keys (k <= 31).

    key = digits e[k-1..0], e[k]; the forward packing F = sum e[i] 4^i is
    the key rotated right by one base."""
    kb = 2 * (k + 1)
    x = keys.astype(np.uint64)
    mask = np.uint64((1 << kb) - 1) if kb < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    F = (x >> np.uint64(2)) | ((x & np.uint64(3)) << np.uint64(kb - 2))
    # reverse the k+1 two-bit groups and complement
    R = np.zeros_like(F)
    t = F.copy()
    for _ in range(k + 1):
        R = (R << np.uint64(2)) | (np.uint64(3) - (t & np.uint64(3)))
        t >>= np.uint64(2)
    R &= mask
    return (((R << np.uint64(2)) & mask) | (R >> np.uint64(kb - 2))).astype(np.uint64)


def graph_invariants(h, n_edges: int, rc_closed: bool = True):
    """Properties that hold for any SdBG built by the reading used here."""
    m = h.m
    assert int(h.F[5]) == m and int(h.F[0]) == 0 and int(h.F[1]) == 0
    assert all(int(h.F[i]) <= int(h.F[i + 1]) for i in range(5))
    assert popcount(h.valid) == n_edges
    assert popcount(h.tip) == h.t
    if rc_closed:
        assert m == n_edges + 2 * h.t
    last = bits(h.last, m)
    tip = bits(h.tip, m)
    valid = bits(h.valid, m)
    assert m == 0 or last[-1]
    assert not (tip & valid).any()
    lab = h.W & 7
    minus = (h.W >> 3) & 1
    assert (lab <= 4).all()
    assert not minus[lab == 0].any() and not minus[tip].any()
    assert (h.mult[~valid] == 0).all() and (h.mult[valid] >= 1).all()
    # nodes: runs closed by a last bit; a node is a tip node iff its rows are tips
    node_end = np.flatnonzero(last)
    node_start = np.concatenate([[0], node_end[:-1] + 1]) if len(node_end) else np.zeros(0, dtype=np.int64)
    assert (tip[node_start] == tip[node_end]).all()
    F = h.F.astype(np.int64)
    for c in range(1, 5):
        in_block = (node_start >= F[c]) & (node_start < F[c + 1])
        nontip_nodes = int((in_block & ~tip[node_start]).sum())
        unflagged_c = int(((lab == c) & (minus == 0)).sum())
        assert unflagged_c == nontip_nodes, f"block {c}: {unflagged_c} unflagged rows vs {nontip_nodes} nodes"
