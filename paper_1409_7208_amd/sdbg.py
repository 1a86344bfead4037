"""ctypes binding of libsdbg.so (the C ABI declared in include/sdbg.h).

Argument marshalling only: every step of the construction runs in the HIP
library.  Device inputs are torch tensors (torch supplies device memory and
streams); host inputs are numpy arrays.  There is no CPU fallback: if the
library is missing, loading fails with an error.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdbg.so")

SDBG_OK = 0
# fixed device scratch of the allocation-free counting call (SDBG_NOALLOC_SCRATCH_MB)
NOALLOC_SCRATCH_BYTES = 256 << 20


class SdbgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sdbg error {code}: {msg}")
        self.code = code


class _Reads(ctypes.Structure):
    _fields_ = [
        ("seq", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
        ("n_reads", ctypes.c_uint64),
        ("on_device", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("d", ctypes.c_uint32),
        ("mercy", ctypes.c_uint32),
        ("prefix_len", ctypes.c_uint32),
        ("mem_budget", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
    ]


class _Edges(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("w", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("n_mercy", ctypes.c_uint64),
        ("n_occ", ctypes.c_uint64),
        ("keys", ctypes.c_void_p),
        ("count", ctypes.c_void_p),
    ]


class _Graph(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("w", ctypes.c_uint32),
        ("m", ctypes.c_uint64),
        ("t", ctypes.c_uint64),
        ("W", ctypes.c_void_p),
        ("last", ctypes.c_void_p),
        ("valid", ctypes.c_void_p),
        ("tip", ctypes.c_void_p),
        ("mult", ctypes.c_void_p),
        ("F", ctypes.c_uint64 * 6),
        ("tip_seq", ctypes.c_void_p),
        ("tip_words", ctypes.c_uint64),
    ]


class _Unitigs(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("n_cycles", ctypes.c_uint64),
        ("n_bases", ctypes.c_uint64),
        ("first_row", ctypes.c_void_p),
        ("len", ctypes.c_void_p),
        ("mult", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
        ("seq", ctypes.c_void_p),
    ]


_lib = None


def load(path: str | None = None):
    """Loads libsdbg.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run paper_1409_7208_amd/build.py (or __graft_entry__.build())")
    # torch ships its own HIP runtime (same soname).  Load it first so that
    # the library binds to that copy: two HIP/HSA runtimes in one process do
    # not share the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    lib.sdbg_count_solid.argtypes = [P(_Reads), P(_Params), P(P(_Edges))]
    lib.sdbg_count_solid.restype = ctypes.c_int
    lib.sdbg_build.argtypes = [P(_Edges), P(_Params), P(P(_Graph))]
    lib.sdbg_build.restype = ctypes.c_int
    lib.sdbg_batch_run.argtypes = [P(_Reads), ctypes.c_uint64, P(_Params), P(P(_Edges)), P(P(_Graph))]
    lib.sdbg_batch_run.restype = ctypes.c_int
    lib.sdbg_edges_from_host.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, P(P(_Edges))]
    lib.sdbg_edges_from_host.restype = ctypes.c_int
    lib.sdbg_edges_to_host.argtypes = [P(_Edges), ctypes.c_void_p, ctypes.c_void_p]
    lib.sdbg_edges_to_host.restype = ctypes.c_int
    lib.sdbg_graph_to_host.argtypes = [P(_Graph)] + [ctypes.c_void_p] * 6
    lib.sdbg_graph_to_host.restype = ctypes.c_int
    lib.sdbg_free.argtypes = [ctypes.c_void_p]
    lib.sdbg_free.restype = None
    lib.sdbg_last_error.argtypes = []
    lib.sdbg_last_error.restype = ctypes.c_char_p
    lib.sdbg_trim.argtypes = []
    lib.sdbg_trim.restype = None
    lib.sdbg_profile_enable.argtypes = [ctypes.c_int]
    lib.sdbg_profile_enable.restype = None
    lib.sdbg_profile_reset.argtypes = []
    lib.sdbg_profile_reset.restype = None
    lib.sdbg_profile_count.argtypes = []
    lib.sdbg_profile_count.restype = ctypes.c_uint32
    lib.sdbg_profile_get.argtypes = [ctypes.c_uint32, P(ctypes.c_char_p), P(ctypes.c_double), P(ctypes.c_uint64)]
    lib.sdbg_profile_get.restype = ctypes.c_int
    lib.sdbg_pool_stats.argtypes = [P(ctypes.c_uint64)] * 3 + [ctypes.c_int]
    lib.sdbg_pool_stats.restype = ctypes.c_int
    lib.sdbg_fail_alloc_after.argtypes = [ctypes.c_int64]
    lib.sdbg_fail_alloc_after.restype = ctypes.c_int
    _lib = lib
    return lib


def _unitig_api():
    """The library with the unitig calls' signatures declared (pointers
    must not pass through ctypes' default int conversion)."""
    lib = load()
    if not getattr(lib, "_unitig_api", False):
        P = ctypes.POINTER
        lib.sdbg_unitigs_build.argtypes = [P(_Graph), ctypes.c_void_p, P(P(_Unitigs)), ctypes.c_void_p]
        lib.sdbg_unitigs_build.restype = ctypes.c_int
        lib.sdbg_unitigs_to_host.argtypes = [P(_Unitigs)] + [ctypes.c_void_p] * 5
        lib.sdbg_unitigs_to_host.restype = ctypes.c_int
        lib._unitig_api = True
    return lib


def _check(rc: int):
    if rc != SDBG_OK:
        raise SdbgError(rc, load().sdbg_last_error().decode(errors="replace"))


def pool_stats(reset_peak: bool = False) -> dict:
    """Device bytes of the library's pool on the current device: in use,
    peak since the last reset, cached."""
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().sdbg_pool_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 1 if reset_peak else 0))
    return {"in_use": a.value, "peak": b.value, "cached": c.value}


def fail_alloc_after(after: int):
    """Test hook: the pool allocation after `after` more successful ones
    fails once (negative: off)."""
    _check(load().sdbg_fail_alloc_after(after))


def key_words(k: int) -> int:
    return (2 * (k + 1) + 63) // 64


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Edges:
    """Edge set E in device memory (owned; freed by close() or on GC)."""

    def __init__(self, ptr):
        self._p = ptr

    @property
    def raw(self) -> _Edges:
        return self._p.contents

    k = property(lambda s: s.raw.k)
    w = property(lambda s: s.raw.w)
    n = property(lambda s: s.raw.n)
    n_mercy = property(lambda s: s.raw.n_mercy)
    n_occ = property(lambda s: s.raw.n_occ)

    def to_host(self) -> tuple[np.ndarray, np.ndarray]:
        r = self.raw
        keys = np.zeros(r.n * r.w + 1, dtype=np.uint64)
        cnt = np.zeros(r.n + 1, dtype=np.uint32)
        _check(load().sdbg_edges_to_host(self._p, keys.ctypes.data, cnt.ctypes.data))
        return keys[: r.n * r.w].reshape(r.n, r.w), cnt[: r.n]

    def close(self):
        if self._p:
            load().sdbg_free(ctypes.cast(self._p, ctypes.c_void_p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class HostGraph:
    k: int
    m: int
    t: int
    W: np.ndarray
    last: np.ndarray
    valid: np.ndarray
    tip: np.ndarray
    mult: np.ndarray
    F: np.ndarray
    tip_seq: np.ndarray


class Graph:
    """SdBG arrays in device memory (owned)."""

    def __init__(self, ptr):
        self._p = ptr

    @property
    def raw(self) -> _Graph:
        return self._p.contents

    m = property(lambda s: s.raw.m)
    t = property(lambda s: s.raw.t)

    @property
    def F(self) -> np.ndarray:
        return np.array(list(self.raw.F), dtype=np.uint64)

    def to_host(self) -> HostGraph:
        r = self.raw
        words = (r.m + 63) // 64
        W = np.zeros(r.m + 1, dtype=np.uint8)
        last = np.zeros(words + 1, dtype=np.uint64)
        valid = np.zeros(words + 1, dtype=np.uint64)
        tip = np.zeros(words + 1, dtype=np.uint64)
        mult = np.zeros(r.m + 1, dtype=np.uint32)
        ts = np.zeros(r.tip_words + 1, dtype=np.uint64)
        _check(load().sdbg_graph_to_host(self._p, W.ctypes.data, last.ctypes.data, valid.ctypes.data, tip.ctypes.data,
                                         mult.ctypes.data, ts.ctypes.data))
        return HostGraph(r.k, r.m, r.t, W[: r.m], last[:words], valid[:words], tip[:words], mult[: r.m], self.F,
                         ts[: r.tip_words])

    def close(self):
        if self._p:
            load().sdbg_free(ctypes.cast(self._p, ctypes.c_void_p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class DeviceReads:
    """A read set already in device memory, given by raw pointers (e.g. the
    unitigs of a graph); `owner` keeps the memory alive."""

    seq_ptr: int | None
    offsets_ptr: int
    n_reads: int
    owner: object = None


def _reads_struct(seq, offsets):
    """torch device tensors -> device pointers; numpy -> host pointers."""
    keep = []
    if isinstance(seq, DeviceReads):
        return _Reads(seq.seq_ptr, seq.offsets_ptr, seq.n_reads, 1, 0), [seq]
    if hasattr(seq, "data_ptr"):
        assert seq.is_cuda and offsets.is_cuda, "torch inputs must be device tensors"
        assert seq.dtype.itemsize == 1 and offsets.dtype.itemsize == 8
        assert seq.is_contiguous() and offsets.is_contiguous()
        n_reads = offsets.numel() - 1
        r = _Reads(seq.data_ptr() if seq.numel() else None, offsets.data_ptr(), n_reads, 1, 0)
    else:
        s = np.ascontiguousarray(seq, dtype=np.uint8)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        keep += [s, o]
        r = _Reads(s.ctypes.data if s.size else None, o.ctypes.data, o.shape[0] - 1, 0, 0)
    return r, keep


def count_solid(seq, offsets, k: int, d: int = 2, mercy: bool = False, prefix_len: int = 8, mem_budget: int = 0,
                stream=None) -> Edges:
    lib = load()
    r, keep = _reads_struct(seq, offsets)
    p = _Params(k, d, 1 if mercy else 0, prefix_len, mem_budget, _stream_ptr(stream))
    out = ctypes.POINTER(_Edges)()
    _check(lib.sdbg_count_solid(ctypes.byref(r), ctypes.byref(p), ctypes.byref(out)))
    del keep
    return Edges(out)


def count_solid_noalloc(seq, offsets, k: int, d: int, mercy: bool, keys_out, count_out, prefix_len: int = 8,
                        mem_budget: int = 0, stream=None) -> dict:
    """Allocation-free counting into caller buffers: keys_out (device uint64
    tensor of cap*w words) and count_out (device int32/uint32 tensor of cap
    entries).  Returns n, n_mercy, n_occ and scratch_peak."""
    lib = load()
    if not getattr(lib, "_noalloc_api", False):
        P = ctypes.POINTER
        lib.sdbg_count_solid_noalloc.argtypes = [P(_Reads), P(_Params), ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_uint64] + [P(ctypes.c_uint64)] * 4
        lib.sdbg_count_solid_noalloc.restype = ctypes.c_int
        lib._noalloc_api = True
    assert keys_out.is_cuda and count_out.is_cuda and keys_out.is_contiguous() and count_out.is_contiguous()
    assert keys_out.dtype.itemsize == 8 and count_out.dtype.itemsize == 4
    w = key_words(k)
    cap = min(keys_out.numel() // w, count_out.numel())
    r, keep = _reads_struct(seq, offsets)
    p = _Params(k, d, 1 if mercy else 0, prefix_len, mem_budget, _stream_ptr(stream))
    n, nm, no, peak = (ctypes.c_uint64() for _ in range(4))
    rc = lib.sdbg_count_solid_noalloc(ctypes.byref(r), ctypes.byref(p), keys_out.data_ptr(), count_out.data_ptr(),
                                      cap, ctypes.byref(n), ctypes.byref(nm), ctypes.byref(no), ctypes.byref(peak))
    del keep
    if rc != SDBG_OK:
        err = SdbgError(rc, lib.sdbg_last_error().decode(errors="replace"))
        err.n = n.value
        raise err
    return {"n": n.value, "n_mercy": nm.value, "n_occ": no.value, "scratch_peak": peak.value}


def build(edges: Edges, stream=None) -> Graph:
    lib = load()
    p = _Params(edges.k, 0, 0, 0, 0, _stream_ptr(stream))
    out = ctypes.POINTER(_Graph)()
    _check(lib.sdbg_build(edges._p, ctypes.byref(p), ctypes.byref(out)))
    return Graph(out)


NAV_NODE, NAV_FORWARD, NAV_BACKWARD, NAV_OUTDEG, NAV_INDEG, NAV_LABEL = 1, 2, 3, 4, 5, 6


class Index:
    """Navigation index of a graph on the device (sdbg_index_build); the
    graph must outlive it."""

    def __init__(self, graph: Graph, stream=None):
        lib = load()
        if not getattr(lib, "_nav_api", False):
            P = ctypes.POINTER
            lib.sdbg_index_build.argtypes = [P(_Graph), P(_Params), ctypes.POINTER(ctypes.c_void_p)]
            lib.sdbg_index_build.restype = ctypes.c_int
            lib.sdbg_navigate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_void_p]
            lib.sdbg_navigate.restype = ctypes.c_int
            lib._nav_api = True
        p = _Params(graph.raw.k, 0, 0, 0, 0, _stream_ptr(stream))
        h = ctypes.c_void_p()
        _check(lib.sdbg_index_build(graph._p, ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.k = graph.raw.k
        self._graph = graph

    def navigate(self, op: int, rows, out, stream=None):
        """rows: device uint64/int64 tensor; out: device tensor of n words
        (n * ceil(2k/64) for NAV_LABEL)."""
        assert rows.is_cuda and out.is_cuda and rows.is_contiguous() and out.is_contiguous()
        _check(load().sdbg_navigate(self._h, op, rows.data_ptr(), rows.numel(), out.data_ptr(), _stream_ptr(stream)))

    def remove_tips(self, max_len: int, stream=None) -> int:
        """Clears the valid bits of the tips of the indexed graph (paths of
        at most max_len edges, sdbg_remove_tips); returns how many."""
        lib = load()
        if not getattr(lib, "_tips_api", False):
            lib.sdbg_remove_tips.argtypes = [ctypes.POINTER(_Graph), ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]
            lib.sdbg_remove_tips.restype = ctypes.c_int
            lib._tips_api = True
        n = ctypes.c_uint64()
        _check(lib.sdbg_remove_tips(self._graph._p, self._h, max_len, ctypes.byref(n), _stream_ptr(stream)))
        return n.value

    def unitigs(self, stream=None) -> "Unitigs":
        """Unitigs of the indexed graph's valid edges (sdbg_unitigs_build)."""
        lib = _unitig_api()
        out = ctypes.POINTER(_Unitigs)()
        _check(lib.sdbg_unitigs_build(self._graph._p, self._h, ctypes.byref(out), _stream_ptr(stream)))
        return Unitigs(out)

    def merge_bubbles(self, unitigs: "Unitigs", max_len: int, stream=None) -> int:
        """Removes all but the best branch of every bubble of unitigs of at
        most max_len edges (sdbg_merge_bubbles); returns the edges removed.
        unitigs must be those of the graph's current valid edges."""
        return self._clean(unitigs, max_len, None, stream)

    def remove_low_coverage(self, unitigs: "Unitigs", max_len: int, ratio_permille: int, stream=None) -> int:
        """Removes unitigs of at most max_len edges whose mean multiplicity
        is below ratio_permille / 1000 of their neighbouring edges' mean
        (sdbg_remove_low_coverage); returns the edges removed."""
        return self._clean(unitigs, max_len, ratio_permille, stream)

    def _clean(self, unitigs, max_len, ratio_permille, stream):
        lib = _unitig_api()
        if not getattr(lib, "_clean_api", False):
            P = ctypes.POINTER
            lib.sdbg_merge_bubbles.argtypes = [P(_Graph), ctypes.c_void_p, P(_Unitigs), ctypes.c_uint32,
                                               P(ctypes.c_uint64), ctypes.c_void_p]
            lib.sdbg_merge_bubbles.restype = ctypes.c_int
            lib.sdbg_remove_low_coverage.argtypes = [P(_Graph), ctypes.c_void_p, P(_Unitigs), ctypes.c_uint32,
                                                     ctypes.c_uint32, P(ctypes.c_uint64), ctypes.c_void_p]
            lib.sdbg_remove_low_coverage.restype = ctypes.c_int
            lib._clean_api = True
        n = ctypes.c_uint64()
        if ratio_permille is None:
            rc = lib.sdbg_merge_bubbles(self._graph._p, self._h, unitigs._p, max_len, ctypes.byref(n),
                                        _stream_ptr(stream))
        else:
            rc = lib.sdbg_remove_low_coverage(self._graph._p, self._h, unitigs._p, max_len, ratio_permille,
                                              ctypes.byref(n), _stream_ptr(stream))
        _check(rc)
        return n.value

    def close(self):
        if self._h:
            load().sdbg_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class HostUnitigs:
    k: int
    n_cycles: int
    first_row: np.ndarray
    len: np.ndarray
    mult: np.ndarray
    offsets: np.ndarray
    seq: np.ndarray  # bytes 'A', 'C', 'G', 'T'

    def sequence(self, u: int) -> str:
        return self.seq[self.offsets[u] : self.offsets[u + 1]].tobytes().decode()


class Unitigs:
    """Unitigs of a graph in device memory (owned)."""

    def __init__(self, ptr):
        self._p = ptr

    @property
    def raw(self) -> _Unitigs:
        return self._p.contents

    n = property(lambda s: s.raw.n)
    n_cycles = property(lambda s: s.raw.n_cycles)
    n_bases = property(lambda s: s.raw.n_bases)

    def to_host(self) -> HostUnitigs:
        r = self.raw
        a = [np.zeros(r.n + 1, dtype=np.uint64) for _ in range(3)]
        off = np.zeros(r.n + 1, dtype=np.uint64)
        seq = np.zeros(r.n_bases + 1, dtype=np.uint8)
        _check(_unitig_api().sdbg_unitigs_to_host(self._p, a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data,
                                           off.ctypes.data, seq.ctypes.data))
        return HostUnitigs(r.k, r.n_cycles, a[0][: r.n], a[1][: r.n], a[2][: r.n], off, seq[: r.n_bases])

    def as_reads(self) -> DeviceReads:
        """The unitigs as a device read set (for counting at another k)."""
        r = self.raw
        return DeviceReads(r.seq if r.n_bases else None, r.offsets, r.n, self)

    def close(self):
        if self._p:
            load().sdbg_free(ctypes.cast(self._p, ctypes.c_void_p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def edges_union(a: Edges, b: Edges, stream=None) -> Edges:
    """Keys of either edge set with summed counts (sdbg_edges_union)."""
    lib = load()
    if not getattr(lib, "_union_api", False):
        P = ctypes.POINTER
        lib.sdbg_edges_union.argtypes = [P(_Edges), P(_Edges), P(_Params), P(P(_Edges))]
        lib.sdbg_edges_union.restype = ctypes.c_int
        lib._union_api = True
    p = _Params(a.k, 0, 0, 0, 0, _stream_ptr(stream))
    out = ctypes.POINTER(_Edges)()
    _check(lib.sdbg_edges_union(a._p, b._p, ctypes.byref(p), ctypes.byref(out)))
    return Edges(out)


class _Clean(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("tip_factor", "bubble_factor", "low_cov_factor", "low_cov_permille")]


def multi_k(seq, offsets, ks, d: int = 2, mercy: bool = True, tip_factor: int = 2, bubble_factor: int = 2,
            low_cov_factor: int = 2, low_cov_permille: int = 200, prefix_len: int = 8, mem_budget: int = 0,
            stream=None) -> tuple[Unitigs, np.ndarray]:
    """Graphs from the smallest k to the largest, each cleaned (tips,
    bubbles, low local coverage; limits in multiples of k, 0 skips a step),
    the unitigs of one k counted into the next (sdbg_multi_k).  Returns the
    last k's unitigs and per-k stats (edges, edges added by the unitigs,
    edges removed as tips, in bubbles and for low coverage, unitigs)."""
    lib = load()
    if not getattr(lib, "_multik_api", False):
        P = ctypes.POINTER
        lib.sdbg_multi_k.argtypes = [P(_Reads), ctypes.c_void_p, ctypes.c_uint32, P(_Params), P(_Clean),
                                     ctypes.c_void_p, P(P(_Unitigs))]
        lib.sdbg_multi_k.restype = ctypes.c_int
        lib._multik_api = True
    r, keep = _reads_struct(seq, offsets)
    kk = np.ascontiguousarray(ks, dtype=np.uint32)
    stats = np.zeros(6 * len(kk), dtype=np.uint64)
    p = _Params(0, d, 1 if mercy else 0, prefix_len, mem_budget, _stream_ptr(stream))
    cl = _Clean(tip_factor, bubble_factor, low_cov_factor, low_cov_permille)
    out = ctypes.POINTER(_Unitigs)()
    _check(lib.sdbg_multi_k(ctypes.byref(r), kk.ctypes.data, len(kk), ctypes.byref(p), ctypes.byref(cl),
                            stats.ctypes.data, ctypes.byref(out)))
    del keep
    return Unitigs(out), stats.reshape(len(kk), 6)


class _Bwt(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("n_reads", ctypes.c_uint64), ("bwt", ctypes.c_void_p),
                ("sa", ctypes.c_void_p)]


def read_bwt(seq, offsets, stream=None, to_host: bool = True):
    """Multi-string BWT of a read set (sdbg_read_bwt): returns (bwt bytes,
    suffix array of text positions), copied to the host; with to_host False
    the result is released on the device and only its length returned."""
    lib = load()
    if not getattr(lib, "_bwt_api", False):
        P = ctypes.POINTER
        lib.sdbg_read_bwt.argtypes = [P(_Reads), P(_Params), P(P(_Bwt))]
        lib.sdbg_read_bwt.restype = ctypes.c_int
        lib.sdbg_bwt_to_host.argtypes = [P(_Bwt), ctypes.c_void_p, ctypes.c_void_p]
        lib.sdbg_bwt_to_host.restype = ctypes.c_int
        lib._bwt_api = True
    r, keep = _reads_struct(seq, offsets)
    p = _Params(0, 0, 0, 0, 0, _stream_ptr(stream))
    out = ctypes.POINTER(_Bwt)()
    _check(lib.sdbg_read_bwt(ctypes.byref(r), ctypes.byref(p), ctypes.byref(out)))
    del keep
    try:
        n = out.contents.n
        if not to_host:
            return n
        b = np.zeros(n + 1, dtype=np.uint8)
        sa = np.zeros(n + 1, dtype=np.uint64)
        _check(lib.sdbg_bwt_to_host(out, b.ctypes.data, sa.ctypes.data))
    finally:
        lib.sdbg_free(ctypes.cast(out, ctypes.c_void_p))
    return b[:n], sa[:n]


def batch_run(sets, k: int, d: int = 2, mercy: bool = False, build: bool = True, prefix_len: int = 8,
              mem_budget: int = 0, stream=None) -> list[tuple[Edges, Graph | None]]:
    """Batched form: sets is a sequence of (seq, offsets) pairs (device
    tensors or host arrays).  Returns one (Edges, Graph or None) per set."""
    lib = load()
    n = len(sets)
    arr = (_Reads * max(n, 1))()
    keep = []
    for i, (seq, off) in enumerate(sets):
        r, kp = _reads_struct(seq, off)
        arr[i] = r
        keep += kp
    p = _Params(k, d, 1 if mercy else 0, prefix_len, mem_budget, _stream_ptr(stream))
    eo = (ctypes.POINTER(_Edges) * max(n, 1))()
    go = (ctypes.POINTER(_Graph) * max(n, 1))()
    _check(lib.sdbg_batch_run(arr, n, ctypes.byref(p), eo, go if build else None))
    del keep
    return [(Edges(eo[i]), Graph(go[i]) if build else None) for i in range(n)]


class _Tune(ctypes.Structure):
    _fields_ = [
        ("digit_bits", ctypes.c_uint32),
        ("tile_shift", ctypes.c_uint32),
        ("leaf_wg_per_cu", ctypes.c_uint32),
        ("leaf_cap_shift", ctypes.c_uint32),
        ("first_bits", ctypes.c_uint32),
        ("mercy_shift", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 2),
    ]


def _tune_api(lib):
    if getattr(lib, "_tune_api", False):
        return
    P = ctypes.POINTER
    lib.sdbg_tune_get.argtypes = [P(_Tune)]
    lib.sdbg_tune_get.restype = ctypes.c_int
    lib.sdbg_tune_set.argtypes = [P(_Tune)]
    lib.sdbg_tune_set.restype = ctypes.c_int
    lib.sdbg_autotune.argtypes = [P(_Reads), ctypes.c_uint64, P(_Params), ctypes.c_uint32, P(_Tune)]
    lib.sdbg_autotune.restype = ctypes.c_int
    lib._tune_api = True


def tune_get() -> dict:
    lib = load()
    _tune_api(lib)
    t = _Tune()
    _check(lib.sdbg_tune_get(ctypes.byref(t)))
    return _tune_dict(t)


def _tune_dict(t) -> dict:
    return {"digit_bits": t.digit_bits, "tile_shift": t.tile_shift, "leaf_wg_per_cu": t.leaf_wg_per_cu,
            "leaf_cap_shift": t.leaf_cap_shift, "first_bits": t.first_bits, "mercy_shift": t.mercy_shift}


def tune_set(t: dict | None = None):
    """Sets the engine's launch parameters (None restores the defaults)."""
    lib = load()
    _tune_api(lib)
    if t is None:
        _check(lib.sdbg_tune_set(None))
    else:
        full = tune_get()
        full.update(t)
        x = _Tune()
        for key, val in full.items():
            setattr(x, key, int(val))
        _check(lib.sdbg_tune_set(ctypes.byref(x)))


def autotune(sets, k: int, d: int = 2, mercy: bool = False, reps: int = 3) -> dict:
    """Picks the fastest launch parameters on a sample of read sets (the
    batched count) and leaves them in effect."""
    lib = load()
    _tune_api(lib)
    n = len(sets)
    arr = (_Reads * max(n, 1))()
    keep = []
    for i, (seq, off) in enumerate(sets):
        r, kp = _reads_struct(seq, off)
        arr[i] = r
        keep += kp
    p = _Params(k, d, 1 if mercy else 0, 8, 0, None)
    t = _Tune()
    _check(lib.sdbg_autotune(arr, n, ctypes.byref(p), reps, ctypes.byref(t)))
    del keep
    return _tune_dict(t)


def edges_from_host(keys: np.ndarray, counts: np.ndarray, k: int) -> Edges:
    lib = load()
    w = key_words(k)
    kk = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1, w)
    cc = np.ascontiguousarray(counts, dtype=np.uint32)
    out = ctypes.POINTER(_Edges)()
    _check(lib.sdbg_edges_from_host(kk.ctypes.data if kk.size else None, cc.ctypes.data if cc.size else None,
                                    kk.shape[0], k, ctypes.byref(out)))
    return Edges(out)


def trim():
    load().sdbg_trim()


def profile_enable(on: bool = True):
    load().sdbg_profile_enable(1 if on else 0)


def profile_reset():
    load().sdbg_profile_reset()


def profile_records() -> list[tuple[str, float, int]]:
    """(kernel name, ms, algorithmic bytes) per profiled launch."""
    lib = load()
    out = []
    for i in range(lib.sdbg_profile_count()):
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        b = ctypes.c_uint64()
        _check(lib.sdbg_profile_get(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(b)))
        out.append((name.value.decode(), ms.value, b.value))
    return out


class _ServerCfg(ctypes.Structure):
    _fields_ = [
        ("max_jobs", ctypes.c_uint32),
        ("queue_cap", ctypes.c_uint32),
        ("mem_budget", ctypes.c_uint64),
        ("build", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class _JobStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
        ("submit_s", ctypes.c_double),
        ("start_s", ctypes.c_double),
        ("end_s", ctypes.c_double),
        ("n_occ", ctypes.c_uint64),
        ("footprint", ctypes.c_uint64),
    ]


@dataclasses.dataclass
class JobResult:
    status: int  # 0 done, 1 waiting, 2 running, < 0 error code
    edges: Edges | None
    graph: Graph | None
    submit_s: float
    start_s: float
    end_s: float
    n_occ: int
    footprint: int
    error: str = ""


def _server_api(lib):
    if getattr(lib, "_server_api", False):
        return
    P = ctypes.POINTER
    lib.sdbg_server_start.argtypes = [P(_ServerCfg), ctypes.c_void_p]
    lib.sdbg_server_start.restype = ctypes.c_int
    lib.sdbg_server_submit.argtypes = [ctypes.c_void_p, P(_Reads), P(_Params), P(ctypes.c_uint64)]
    lib.sdbg_server_submit.restype = ctypes.c_int
    lib.sdbg_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, P(P(_Edges)), P(P(_Graph)),
                                     P(_JobStats)]
    lib.sdbg_server_poll.restype = ctypes.c_int
    lib.sdbg_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.sdbg_server_cancel.restype = ctypes.c_int
    lib.sdbg_server_stop.argtypes = [ctypes.c_void_p]
    lib.sdbg_server_stop.restype = ctypes.c_int
    lib.sdbg_server_state.argtypes = [ctypes.c_void_p, P(_ServerInfo)]
    lib.sdbg_server_state.restype = ctypes.c_int
    lib.sdbg_server_trace.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(ctypes.c_char_p), P(ctypes.c_char_p),
                                      P(ctypes.c_double)]
    lib.sdbg_server_trace.restype = ctypes.c_int
    lib.sdbg_job_footprint.argtypes = [P(_Reads), P(_Params), P(ctypes.c_uint64)]
    lib.sdbg_job_footprint.restype = ctypes.c_int
    lib._server_api = True


class _ServerInfo(ctypes.Structure):
    _fields_ = [
        ("budget", ctypes.c_uint64),
        ("mem_in_use", ctypes.c_uint64),
        ("queued", ctypes.c_uint32),
        ("running", ctypes.c_uint32),
        ("jobs", ctypes.c_uint64),
        ("uptime_s", ctypes.c_double),
    ]


def job_footprint(seq, offsets, k: int, d: int = 2, mercy: bool = True, prefix_len: int = 8) -> int:
    """Device bytes the request loop reserves for a job on these host reads."""
    lib = load()
    _server_api(lib)
    r, keep = _reads_struct(seq, offsets)
    p = _Params(k, d, 1 if mercy else 0, prefix_len, 0, None)
    b = ctypes.c_uint64()
    _check(lib.sdbg_job_footprint(ctypes.byref(r), ctypes.byref(p), ctypes.byref(b)))
    del keep
    return b.value


class Server:
    """Served form (sdbg_server_*): a request loop on the current device."""

    def __init__(self, max_jobs: int = 4, queue_cap: int = 0, mem_budget: int = 0, build: bool = True):
        lib = load()
        _server_api(lib)
        cfg = _ServerCfg(max_jobs, queue_cap, mem_budget, 1 if build else 0, 0)
        h = ctypes.c_void_p()
        _check(lib.sdbg_server_start(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, seq, offsets, k: int, d: int = 2, mercy: bool = False, prefix_len: int = 8,
               mem_budget: int = 0) -> int:
        """Queues a job on host reads; raises SdbgError (code -5) if the queue is full."""
        lib = load()
        r, keep = _reads_struct(seq, offsets)
        p = _Params(k, d, 1 if mercy else 0, prefix_len, mem_budget, None)
        jid = ctypes.c_uint64()
        _check(lib.sdbg_server_submit(self._h, ctypes.byref(r), ctypes.byref(p), ctypes.byref(jid)))
        del keep
        return jid.value

    def poll(self, job_id: int, wait: bool = True) -> JobResult:
        lib = load()
        e = ctypes.POINTER(_Edges)()
        g = ctypes.POINTER(_Graph)()
        st = _JobStats()
        rc = lib.sdbg_server_poll(self._h, job_id, 1 if wait else 0, ctypes.byref(e), ctypes.byref(g),
                                  ctypes.byref(st))
        err = "" if rc >= 0 else lib.sdbg_last_error().decode(errors="replace")
        if rc == SDBG_OK:
            return JobResult(0, Edges(e), Graph(g) if g else None, st.submit_s, st.start_s, st.end_s, st.n_occ,
                             st.footprint)
        if rc < 0 and st.status != rc:
            raise SdbgError(rc, err)  # not a job's own result (e.g. unknown id)
        return JobResult(rc, None, None, st.submit_s, st.start_s, st.end_s, st.n_occ, st.footprint, err)

    def state(self) -> dict:
        """Admission budget, footprint bytes in use, queued and running jobs."""
        info = _ServerInfo()
        _check(load().sdbg_server_state(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in _ServerInfo._fields_}

    def trace(self, job_id: int) -> dict:
        """Last kernel stage a running job entered, what it waits on, and
        seconds since either changed."""
        st, act, sec = ctypes.c_char_p(), ctypes.c_char_p(), ctypes.c_double()
        _check(load().sdbg_server_trace(self._h, job_id, ctypes.byref(st), ctypes.byref(act), ctypes.byref(sec)))
        return {"stage": (st.value or b"").decode(), "activity": (act.value or b"").decode(), "seconds": sec.value}

    def cancel(self, job_id: int) -> int:
        return load().sdbg_server_cancel(self._h, job_id)

    def stop(self):
        if self._h:
            _check(load().sdbg_server_stop(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
