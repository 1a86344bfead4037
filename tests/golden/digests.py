"""SHA-256 digests of an edge set and its SdBG arrays, for comparing
full-size runs whose outputs are too large to store.  Arrays are hashed as
their little-endian bytes: keys as n x w uint64 (word 0 most significant),
counts and mult as uint32, W as uint8, the bit vectors and tip_seq as
uint64 words."""

from __future__ import annotations

import hashlib

import numpy as np


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def block_sizes(keys: np.ndarray, k: int) -> list[int]:
    """Edges per block of the key space (the 4 most significant colex
    symbols, 256 blocks) -- localises a mismatch."""
    if keys.shape[0] == 0:
        return [0] * 256
    kb = 2 * (k + 1)
    top_word_bits = kb - 64 * (keys.shape[1] - 1)
    top = (keys[:, 0] >> np.uint64(top_word_bits - 8)).astype(np.int64) if top_word_bits >= 8 else None
    return np.bincount(top, minlength=256).tolist()


def edge_digest(keys: np.ndarray, counts: np.ndarray, n_mercy: int, n_occ: int, k: int) -> dict:
    return {"n": int(keys.shape[0]), "n_mercy": int(n_mercy), "n_occ": int(n_occ),
            "keys": sha(keys.astype(np.uint64)), "counts": sha(counts.astype(np.uint32)),
            "blocks": block_sizes(keys, k)}


def graph_digest(g) -> dict:
    return {"m": int(g.m), "t": int(g.t), "F": [int(x) for x in g.F],
            "W": sha(g.W.astype(np.uint8)), "last": sha(g.last.astype(np.uint64)),
            "valid": sha(g.valid.astype(np.uint64)), "tip": sha(g.tip.astype(np.uint64)),
            "mult": sha(g.mult.astype(np.uint32)), "tip_seq": sha(g.tip_seq.astype(np.uint64))}
