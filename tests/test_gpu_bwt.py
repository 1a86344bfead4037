"""Read-set BWT on the device (sdbg_read_bwt) against the oracle
(oracle/bwt.py): hand-made read sets (a worked example, identical reads,
empty reads, homopolymers that need many doubling rounds, lower case) and
seeded read sets of the workloads' shape (100-150 bp reads with errors,
ragged lengths across several radix tiles), every suffix and every BWT
character; non-base bytes are rejected."""

from __future__ import annotations

import random

import numpy as np
import pytest

from gpu_util import say
from oracle import bwt as ob
from paper_1409_7208_amd import sdbg, synth

pytestmark = pytest.mark.gpu


def _as_arrays(reads):
    seq = np.frombuffer("".join(reads).encode(), dtype=np.uint8).copy()
    off = np.zeros(len(reads) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    return seq, off


def _check(reads, device=False):
    seq, off = _as_arrays(reads)
    if device:
        import torch

        seq, off = torch.from_numpy(seq).to("cuda"), torch.from_numpy(off.view(np.int64)).to("cuda")
    b, sa = sdbg.read_bwt(seq, off)
    order, want = ob.read_bwt(reads)
    starts = np.array([sum(len(x) for x in reads[:r]) + r for r in range(len(reads))], dtype=np.int64)
    got = [(int(r), int(p - starts[r])) for p in sa.astype(np.int64) for r in [np.searchsorted(starts, p, "right") - 1]]
    assert got == order
    assert b.tobytes().decode() == want
    return len(want)


def test_hand_made_read_sets():
    assert _check(["ACG"]) == 4
    _check(["AC", "AC"])
    _check(["", "A", "", "AC", "ACGT" * 9, ""])
    _check(["A" * 90, "A" * 89, "A" * 90, "AAAAT", "TAAAA" * 20])  # long runs: many rounds
    _check(["acgtNacg".replace("N", "a"), "ACGTAACG"])  # lower case equals upper case
    _check([""])


def test_random_read_sets():
    rng = random.Random(7)
    for trial in range(8):
        g = "".join(rng.choice("ACGT") for _ in range(rng.randint(50, 3000)))
        reads = []
        for _ in range(rng.randint(1, 400)):
            i = rng.randrange(len(g))
            x = list(g[i : i + rng.randint(0, 150)])
            for q in range(len(x)):
                if rng.random() < 0.01:
                    x[q] = rng.choice("ACGT")
            reads.append("".join(x))
        n = _check(reads, device=trial % 2 == 1)
        say(f"trial {trial}: {len(reads)} reads, {n} suffixes")


@pytest.mark.parametrize("n_reads,lo,hi", [(3000, 100, 100), (2000, 60, 150)])
def test_workload_shaped_read_sets(n_reads, lo, hi):
    rs = synth.random_small(n_reads, lo, hi, 20000, 0.005, seed=n_reads)
    reads = [rs.seq[rs.offsets[i] : rs.offsets[i + 1]].tobytes().decode() for i in range(len(rs.offsets) - 1)]
    n = _check(reads, device=True)
    say(f"{n_reads} reads of {lo}-{hi} bp: {n} suffixes ({n // 2048 + 1} radix tiles)")


def test_non_base_bytes_are_rejected():
    seq, off = _as_arrays(["ACGT", "ACNT"])
    with pytest.raises(sdbg.SdbgError):
        sdbg.read_bwt(seq, off)
