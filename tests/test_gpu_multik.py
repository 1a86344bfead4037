"""Edge-set union (sdbg_edges_union) and multiple k with contig feedback
(sdbg_multi_k) on the device against the oracle (oracle/multik.py): union of
overlapping and empty sets for one to four key words, the summed-count
overflow error, the read-bridging case of tests/test_multik_oracle.py, and
a seeded metagenome workload over three k values, unitig by unitig."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import say, to_device
from oracle import multik
from paper_1409_7208_amd import sdbg, synth
from test_multik_oracle import _genome, _reads

pytestmark = pytest.mark.gpu


def _edges(keys, cnt, k):
    return sdbg.edges_from_host(np.ascontiguousarray(keys, dtype=np.uint64), np.ascontiguousarray(cnt, dtype=np.uint32), k)


@pytest.mark.parametrize("k", [21, 41, 81, 110])
def test_edges_union(k):
    rs = synth.random_small(800, 60, 160, 4000, 0.01, seed=k)
    half = len(rs.offsets) // 2
    a = oracle.count_solid(rs.seq, rs.offsets[: half + 1], k, 1, False)
    s0 = half - half // 3  # b's reads overlap a's
    b = oracle.count_solid(rs.seq[int(rs.offsets[s0]) :], rs.offsets[s0:] - rs.offsets[s0], k, 1, False)
    want_k, want_c = multik._union(a.keys, a.counts, b.keys, b.counts)
    ea, eb = _edges(a.keys, a.counts, k), _edges(b.keys, b.counts, k)
    e0 = _edges(np.zeros((0, a.keys.shape[1])), np.zeros(0), k)
    for x, y, wk, wc in ((ea, eb, want_k, want_c), (eb, ea, want_k, want_c), (ea, e0, a.keys, a.counts),
                         (e0, e0, a.keys[:0], a.counts[:0])):
        u = sdbg.edges_union(x, y)
        keys, cnt = u.to_host()
        assert np.array_equal(keys, wk) and np.array_equal(cnt, np.asarray(wc, dtype=np.uint32))
        u.close()
    say(f"k={k}: {len(a.counts)} + {len(b.counts)} -> {len(want_c)} edges")
    for x in (ea, eb, e0):
        x.close()


def test_edges_union_count_overflow():
    keys = np.array([[5], [9]], dtype=np.uint64)
    a = _edges(keys, np.array([0xFFFFFFF0, 1]), 21)
    b = _edges(keys[:1], np.array([0x20]), 21)
    with pytest.raises(sdbg.SdbgError):
        sdbg.edges_union(a, b)
    a.close()
    b.close()


def _compare(u, want, want_stats, stats):
    hu = u.to_host()
    got = [(int(hu.len[i]), int(hu.mult[i]), hu.sequence(i)) for i in range(len(hu.len))]
    assert got == [(r[1], r[2], r[3]) for r in want]
    assert np.array_equal(stats, want_stats)


def test_multi_k_bridges_reads():
    import random

    g = _genome(random.Random(3), 300)
    _, seq, off = _reads(g)
    want, wst = multik.multi_k(seq, off, [15, 31], d=1, mercy=False)
    u, st = sdbg.multi_k(seq, off, [15, 31], d=1, mercy=False, bubble_factor=0, low_cov_factor=0)
    _compare(u, want, wst, st)
    u.close()


@pytest.mark.parametrize("ks,clean", [
    ([21, 41, 61], (2, 2, 2, 200)),
    ([31, 81], (2, 0, 0, 0)),
    ([25, 45], (1, 3, 3, 600)),
])
def test_multi_k_workload(ks, clean):
    rs = synth.metagenome(0.002, k=ks[0])
    want, wst = multik.multi_k(rs.seq, rs.offsets, ks, 2, True, *clean)
    seq, off = to_device(rs)
    u, st = sdbg.multi_k(seq, off, ks, d=2, mercy=True, tip_factor=clean[0], bubble_factor=clean[1],
                         low_cov_factor=clean[2], low_cov_permille=clean[3])
    say(f"ks={ks} clean={clean}: per k [edges, from unitigs, tips, bubbles, low cov, unitigs] = {st.tolist()}")
    _compare(u, want, wst, st)
    u.close()
