"""TEST INFRASTRUCTURE ONLY: the CPU oracle for SdBG construction.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The device library never calls it, and it
never calls the device library.

``count_solid`` and ``build`` wrap the plain C++ implementation in
``sdbg_oracle.cpp`` (string-based, std::sort + std::unordered_map) which
follows Section 2 of the paper step by step; ``count_keys`` counts chosen
edges over all reads for sampled checks of large runs.  ``part_count_solid``
and ``part_build_graph`` (``sdbg_oracle_part.cpp``) compute the same outputs
on packed keys, one block of the key space at a time on several threads, for
read sets too large for the string form; the tests pin them to it.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "sdbg_oracle.cpp"), os.path.join(_HERE, "sdbg_oracle_part.cpp")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, *_SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Graph(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_uint64),
        ("t", ctypes.c_uint64),
        ("W", ctypes.POINTER(ctypes.c_uint8)),
        ("last", ctypes.POINTER(ctypes.c_uint64)),
        ("valid", ctypes.POINTER(ctypes.c_uint64)),
        ("tip", ctypes.POINTER(ctypes.c_uint64)),
        ("mult", ctypes.POINTER(ctypes.c_uint32)),
        ("F", ctypes.c_uint64 * 6),
        ("tip_seq", ctypes.POINTER(ctypes.c_uint64)),
        ("tip_words", ctypes.c_uint64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.POINTER
        lib.oracle_count_solid.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
            p(p(ctypes.c_uint64)), p(p(ctypes.c_uint32)), p(ctypes.c_uint64), p(ctypes.c_uint64), p(ctypes.c_uint64),
        ]
        lib.oracle_count_solid.restype = ctypes.c_int
        lib.oracle_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, p(_Graph)]
        lib.oracle_build.restype = ctypes.c_int
        lib.oracle_free_graph.argtypes = [p(_Graph)]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_count_keys.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_int,
        ]
        lib.oracle_count_keys.restype = ctypes.c_int
        lib.oracle_part_count_solid.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
            ctypes.c_int, ctypes.c_uint64, p(p(ctypes.c_uint64)), p(p(ctypes.c_uint32)), p(ctypes.c_uint64),
            p(ctypes.c_uint64), p(ctypes.c_uint64),
        ]
        lib.oracle_part_count_solid.restype = ctypes.c_int
        lib.oracle_part_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_int, p(_Graph)]
        lib.oracle_part_build.restype = ctypes.c_int
        lib.oracle_narrow_count.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)]
        lib.oracle_narrow_count.restype = ctypes.c_int
        _lib = lib
    return _lib


def key_words(k: int) -> int:
    return (2 * (k + 1) + 63) // 64


@dataclasses.dataclass
class Edges:
    k: int
    keys: np.ndarray  # uint64 [n, w], word 0 most significant
    counts: np.ndarray  # uint32 [n]
    n_mercy: int
    n_occ: int


@dataclasses.dataclass
class Graph:
    k: int
    m: int
    t: int
    W: np.ndarray  # uint8 [m]
    last: np.ndarray  # uint64 [ceil(m/64)]
    valid: np.ndarray
    tip: np.ndarray
    mult: np.ndarray  # uint32 [m]
    F: np.ndarray  # uint64 [6]
    tip_seq: np.ndarray  # uint64 [ceil(2kt/64)]


def _as_reads(seq, offsets):
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    return seq, offsets


def _threads(threads):
    return min(16, os.cpu_count() or 1) if threads is None else threads


def count_solid(seq, offsets, k: int, d: int = 2, mercy: bool = False) -> Edges:
    return _count(seq, offsets, k, d, mercy, None)


def part_count_solid(seq, offsets, k: int, d: int = 2, mercy: bool = False, threads: int | None = None,
                     group_keys: int = 0) -> Edges:
    """Same as count_solid, block by block (group_keys: most keys counted
    together, 0 = all)."""
    return _count(seq, offsets, k, d, mercy, (_threads(threads), group_keys))


def _count(seq, offsets, k, d, mercy, part):
    lib = _load()
    seq, offsets = _as_reads(seq, offsets)
    n_reads = offsets.shape[0] - 1
    kp = ctypes.POINTER(ctypes.c_uint64)()
    cp = ctypes.POINTER(ctypes.c_uint32)()
    n = ctypes.c_uint64()
    nm = ctypes.c_uint64()
    nocc = ctypes.c_uint64()
    outs = (ctypes.byref(kp), ctypes.byref(cp), ctypes.byref(n), ctypes.byref(nm), ctypes.byref(nocc))
    sp = seq.ctypes.data if seq.size else None
    if part is None:
        rc = lib.oracle_count_solid(sp, offsets.ctypes.data, n_reads, k, d, int(bool(mercy)), *outs)
    else:
        rc = lib.oracle_part_count_solid(sp, offsets.ctypes.data, n_reads, k, d, int(bool(mercy)), part[0], part[1],
                                         *outs)
    if rc != 0:
        raise ValueError(f"oracle count failed ({rc})")
    w = key_words(k)
    try:
        keys = np.ctypeslib.as_array(kp, shape=(n.value * w + 1,))[: n.value * w].copy().reshape(n.value, w)
        counts = np.ctypeslib.as_array(cp, shape=(n.value + 1,))[: n.value].copy()
    finally:
        lib.oracle_free(ctypes.cast(kp, ctypes.c_void_p))
        lib.oracle_free(ctypes.cast(cp, ctypes.c_void_p))
    return Edges(k, keys, counts, nm.value, nocc.value)


def build_graph(keys: np.ndarray, counts: np.ndarray, k: int) -> Graph:
    return _build(keys, counts, k, None)


def part_build_graph(keys: np.ndarray, counts: np.ndarray, k: int, threads: int | None = None) -> Graph:
    """Same as build_graph, block by block."""
    return _build(keys, counts, k, _threads(threads))


def _build(keys, counts, k, threads):
    lib = _load()
    w = key_words(k)
    keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1, w)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    n = keys.shape[0]
    g = _Graph()
    kp, cp = (keys.ctypes.data if n else None), (counts.ctypes.data if n else None)
    if threads is None:
        rc = lib.oracle_build(kp, cp, n, k, ctypes.byref(g))
    else:
        rc = lib.oracle_part_build(kp, cp, n, k, threads, ctypes.byref(g))
    if rc != 0:
        raise ValueError(f"oracle_build failed ({rc})")
    try:
        m = g.m
        words = (m + 63) // 64
        arr = lambda ptr, cnt: np.ctypeslib.as_array(ptr, shape=(cnt + 1,))[:cnt].copy()
        out = Graph(k, m, g.t, arr(g.W, m), arr(g.last, words), arr(g.valid, words), arr(g.tip, words), arr(g.mult, m),
                    np.array(list(g.F), dtype=np.uint64), arr(g.tip_seq, g.tip_words))
    finally:
        lib.oracle_free_graph(ctypes.byref(g))
    return out


def count_keys(seq, offsets, k: int, qkeys: np.ndarray, threads: int | None = None) -> np.ndarray:
    lib = _load()
    seq, offsets = _as_reads(seq, offsets)
    w = key_words(k)
    q = np.ascontiguousarray(qkeys, dtype=np.uint64).reshape(-1, w)
    out = np.zeros(q.shape[0], dtype=np.uint64)
    threads = _threads(threads)
    rc = lib.oracle_count_keys(seq.ctypes.data if seq.size else None, offsets.ctypes.data, offsets.shape[0] - 1, k,
                               q.ctypes.data if q.size else None, q.shape[0], out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle_count_keys failed ({rc})")
    return out


def narrow_count(c: int) -> int:
    """A count as the oracle reports it (32 bits); raises OverflowError for a
    count of 2^32 or more (the oracle never clamps)."""
    out = ctypes.c_uint32()
    if _load().oracle_narrow_count(c, ctypes.byref(out)) != 0:
        raise OverflowError(f"count {c} does not fit 32 bits")
    return out.value
