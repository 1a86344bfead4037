"""CPU checks of test helpers used by the device tests."""

import numpy as np

import brute
import oracle
from gpu_util import revcomp_keys_w1
from paper_1409_7208_amd import synth


def test_rc_closure_helper_matches_oracle():
    rs = synth.tiny(scale=0.05)
    o = oracle.count_solid(rs.seq, rs.offsets, 21, 2, False)
    k1 = o.keys[:, 0]
    rc = revcomp_keys_w1(k1, 21)
    want = np.array([brute.edge_key(brute.revcomp(brute.key_to_edge(int(x), 21))) for x in k1[:200]], dtype=np.uint64)
    assert np.array_equal(rc[:200], want)
