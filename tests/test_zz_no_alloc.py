"""The allocation-free counting entry point (sdbg_count_solid_noalloc)
against sdbg_count_solid, through the C ABI: identical edge sets (bit-exact)
on two calls in a row, the second with a smaller input, and no device
memory taken by the second call."""

from __future__ import annotations

import numpy as np
import pytest

from gpu_util import say, to_device
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu


def _noalloc(rs, k, d, mercy, cap, device_input=True, mem_budget=0):
    import torch

    seq, off = to_device(rs) if device_input else (rs.seq, rs.offsets)
    w = sdbg.key_words(k)
    keys = torch.zeros(max(cap, 1) * w, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    st = sdbg.count_solid_noalloc(seq, off, k, d, mercy, keys, cnt, mem_budget=mem_budget)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    n = st["n"]
    hk = keys[: n * w].cpu().numpy().view(np.uint64).reshape(n, w)
    hc = cnt[:n].cpu().numpy().view(np.uint32)
    return st, hk, hc, free0 - free1


def _plain(rs, k, d, mercy):
    seq, off = to_device(rs)
    e = sdbg.count_solid(seq, off, k, d, mercy)
    keys, cnt = e.to_host()
    out = (e.n, e.n_mercy, e.n_occ, keys, cnt)
    e.close()
    return out


@pytest.mark.parametrize("k", [21, 41])
def test_noalloc_matches_count_solid_twice(k):
    big = synth.tiny(scale=0.1)
    small = synth.tiny(scale=0.03, seed_extra=1)
    ref_big = _plain(big, k, 2, True)
    ref_small = _plain(small, k, 2, True)
    for name, rs, ref in (("first", big, ref_big), ("second, smaller", small, ref_small)):
        say(f"noalloc k={k} {name}: {rs.n_reads} reads")
        n, n_mercy, n_occ, keys, cnt = ref
        st, hk, hc, taken = _noalloc(rs, k, 2, True, cap=n + 7)
        assert st["n"] == n and st["n_mercy"] == n_mercy and st["n_occ"] == n_occ
        assert np.array_equal(hk, keys)
        assert np.array_equal(hc, cnt)
        assert 0 < st["scratch_peak"] <= sdbg.NOALLOC_SCRATCH_BYTES
        if name != "first":
            assert taken == 0, f"the call took {taken} bytes of device memory"


def test_noalloc_host_input_and_budget():
    rs = synth.tiny(scale=0.05)
    n, n_mercy, n_occ, keys, cnt = _plain(rs, 21, 2, True)
    st, hk, hc, _ = _noalloc(rs, 21, 2, True, cap=n, device_input=False, mem_budget=8 << 20)
    assert st["n"] == n and np.array_equal(hk, keys) and np.array_equal(hc, cnt)


def test_noalloc_rejects_small_output_and_large_input():
    rs = synth.tiny(scale=0.02)
    n = _plain(rs, 21, 2, False)[0]
    with pytest.raises(sdbg.SdbgError) as ei:
        _noalloc(rs, 21, 2, False, cap=n - 1)
    assert ei.value.code == -1 and ei.value.n == n
    # 4 M bases: the size check refuses it before any kernel runs
    big = synth.from_strings(["ACGT" * 25] * 40_000, 21, 2, False)
    with pytest.raises(sdbg.SdbgError) as ei:
        _noalloc(big, 21, 2, False, cap=16)
    assert ei.value.code == -3 and "too large" in str(ei.value)
