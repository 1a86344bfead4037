"""Full-size workloads, in the launch configuration bench.py times.

The oracle cannot build these graphs whole, so the device results are
checked (a) on every output by properties that hold at any size, and (b) on
random samples that the oracle computes one by one: the count of a sampled
edge, and the presence and count of the edge of a sampled read window, by
counting those keys over all reads (oracle.count_keys)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import graph_invariants, say, to_device
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu

CODE = np.full(256, 255, dtype=np.uint8)
for i, ch in enumerate(b"ACGT"):
    CODE[ch] = i
    CODE[ch + 32] = i


def _window_keys(rs, k: int, n: int, rng) -> list[int]:
    """Edge keys of n random windows (reads are ACGT only): digits
    e[k-1], ..., e[0], e[k]."""
    lens = np.diff(rs.offsets.astype(np.int64))
    nw = np.maximum(lens - k, 0)
    reads = rng.choice(np.flatnonzero(nw > 0), size=n)
    out = []
    for r in reads:
        j = int(rng.integers(0, nw[r]))
        s = int(rs.offsets[r]) + j
        e = CODE[rs.seq[s : s + k + 1]].astype(np.int64)
        key = int(e[k])
        for i in range(k):
            key += int(e[i]) << (2 * (i + 1))
        out.append(key)
    return out


def _to_words(keys: list[int], w: int) -> np.ndarray:
    a = np.zeros((len(keys), w), dtype=np.uint64)
    for i, key in enumerate(keys):
        for j in range(w):
            a[i, j] = (key >> (64 * (w - 1 - j))) & 0xFFFFFFFFFFFFFFFF
    return a


def _ascending(keys: np.ndarray) -> bool:
    """Rows (w words, word 0 most significant) strictly ascending."""
    gt = keys[1:, -1] > keys[:-1, -1]
    for j in range(keys.shape[1] - 2, -1, -1):
        gt = (keys[1:, j] > keys[:-1, j]) | ((keys[1:, j] == keys[:-1, j]) & gt)
    return bool(gt.all())


def _find(keys: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Index of each query row in the sorted key rows, or -1."""
    cols = [np.ascontiguousarray(keys[:, j]) for j in range(keys.shape[1])]
    out = np.full(q.shape[0], -1, dtype=np.int64)
    for i in range(q.shape[0]):
        lo, hi = 0, keys.shape[0]
        for j in range(keys.shape[1]):
            col = cols[j][lo:hi]
            a = int(np.searchsorted(col, q[i, j], "left"))
            b = int(np.searchsorted(col, q[i, j], "right"))
            lo, hi = lo + a, lo + b
            if lo == hi:
                break
        if hi - lo == 1:
            out[i] = lo
    return out


def _revcomp(key: int, k: int) -> int:
    e = [(key >> (2 * (i + 1))) & 3 for i in range(k)] + [key & 3]  # e[0..k]
    r = [3 - e[k - i] for i in range(k + 1)]
    out = r[k]
    for i in range(k):
        out += r[i] << (2 * (i + 1))
    return out


def _check_full(rs, k: int, d: int, mercy: bool, n_sample: int = 4000):
    rng = np.random.default_rng(0x14097208 + k)
    w = sdbg.key_words(k)
    seq, off = to_device(rs)
    say(f"full size {rs.name}: {rs.n_reads} reads, k={k}")
    e = sdbg.count_solid(seq, off, k, d, mercy)
    keys, cnt = e.to_host()
    n = keys.shape[0]
    # every output: exact occurrence count, strictly ascending keys within
    # 2(k+1) bits, counts >= d except exactly n_mercy edges below d
    assert e.n_occ == 2 * rs.n_windows(k)
    assert n == 0 or _ascending(keys)
    kb = 2 * (k + 1)
    top_bits = 64 * w - kb
    if top_bits:
        assert int((keys[:, 0] >> np.uint64(64 - top_bits)).max()) == 0
    assert (cnt >= 1).all()
    assert int((cnt < d).sum()) == e.n_mercy
    if not mercy:
        assert e.n_mercy == 0
    # sampled edges: the oracle's count over all reads, and the reverse
    # complement present with the same count
    idx = rng.choice(n, size=min(n_sample, n), replace=False)
    sample = [sum(int(keys[i, j]) << (64 * (w - 1 - j)) for j in range(w)) for i in idx]
    rcs = [_revcomp(x, k) for x in sample]
    oc = oracle.count_keys(rs.seq, rs.offsets, k, _to_words(sample + rcs, w))
    assert np.array_equal(oc[: len(sample)].astype(np.uint32), cnt[idx])
    assert np.array_equal(oc[: len(sample)], oc[len(sample):])
    pos = _find(keys, _to_words(rcs, w))
    assert (pos >= 0).all()
    assert np.array_equal(cnt[pos], cnt[idx])
    # sampled read windows: solid iff counted >= d; then present with that count
    wk = _window_keys(rs, k, n_sample, rng)
    wc = oracle.count_keys(rs.seq, rs.offsets, k, _to_words(wk, w))
    pos = _find(keys, _to_words(wk, w))
    found = pos >= 0
    solid = wc >= d
    assert found[solid].all()
    assert np.array_equal(cnt[pos[solid]], wc[solid].astype(np.uint32))
    assert (cnt[pos[found & ~solid]] == wc[found & ~solid]).all()  # mercy edges keep their count
    say(f"  {n} edges ({e.n_mercy} mercy); sampled windows solid {int(solid.sum())}/{len(wk)}, "
        f"mercy among the others {int((found & ~solid).sum())}")
    # graph: every array by invariants
    g = sdbg.build(e)
    h = g.to_host()
    g.close()
    e.close()
    graph_invariants(h, n)


def test_metagenome_full_size():
    """The bench workload itself: 200 genomes, 10M reads x 100 bp, k = 31,
    d = 2, mercy on, 1.38e9 occurrences."""
    _check_full(synth.metagenome(), 31, 2, True)


def test_large_k_full_size_k61():
    """The large-k workload at k = 61 (two key words): 20M reads x 150 bp,
    3.56e9 occurrences."""
    _check_full(synth.metagenome_long(k=61), 61, 2, True, n_sample=2000)


# ---- element-by-element parity at full size, through digests of every array
import json  # noqa: E402
import os  # noqa: E402
import sys  # noqa: E402

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import digests  # noqa: E402

_GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_digests.json")
_GOLD = json.load(open(_GOLD_PATH)) if os.path.exists(_GOLD_PATH) else {}
_READS: dict = {}


def _full_reads(name: str):
    if name == "metagenome":
        return synth.metagenome(), 31
    k = int(name[4:])
    if "long" not in _READS:  # the same reads at every k
        _READS.clear()
        _READS["long"] = synth.metagenome_long()
    return _READS["long"], k


@pytest.mark.parametrize("name", [n for n in ("metagenome", "long21", "long41", "long61", "long81", "long99")
                                  if n in _GOLD])
def test_full_size_equals_partitioned_oracle(name):
    """Every output of the full-size workloads, bit for bit: SHA-256 digests
    of the keys, counts and every SdBG array (and the edges per key block)
    against those of the partitioned oracle (tests/golden/fullsize_digests.json,
    written by tests/golden/make_fullsize_digests.py)."""
    gold = _GOLD[name]
    rs, k = _full_reads(name)
    say(f"full-size digests {name}: {rs.n_reads} reads, k={k}")
    seq, off = to_device(rs)
    e = sdbg.count_solid(seq, off, k, gold["d"], gold["mercy"])
    del seq, off
    keys, cnt = e.to_host()
    ed = digests.edge_digest(keys, cnt, e.n_mercy, e.n_occ, k)
    del keys, cnt
    for f in ("n", "n_mercy", "n_occ", "blocks", "keys", "counts"):
        assert ed[f] == gold["edges"][f], f
    g = sdbg.build(e)
    e.close()
    h = g.to_host()
    g.close()
    gd = digests.graph_digest(h)
    for f in ("m", "t", "F", "W", "last", "valid", "tip", "mult", "tip_seq"):
        assert gd[f] == gold["graph"][f], f
