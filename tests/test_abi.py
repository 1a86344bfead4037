"""Host-only checks of the C ABI: the library loads, exports every function
include/sdbg.h declares, and rejects invalid arguments before touching a
device.  No compute call is made here."""

from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_1409_7208_amd import sdbg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(sdbg.LIB_PATH):
        from paper_1409_7208_amd import build

        build.build()


def _declared_functions() -> set[str]:
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+(sdbg_[A-Za-z0-9_]+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_exports_every_declared_function():
    _ensure_built()
    declared = _declared_functions()
    assert {"sdbg_count_solid", "sdbg_build", "sdbg_free", "sdbg_last_error"} <= declared
    out = subprocess.run(["nm", "-D", "--defined-only", sdbg.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert declared <= exported, declared - exported
    lib = sdbg.load()
    for name in declared:
        assert hasattr(lib, name)


@pytest.mark.parametrize("k,d,pl,msg", [(1, 2, 8, "k must"), (128, 2, 8, "k must"), (21, 0, 8, "d must"), (21, 2, 9, "prefix_len")])
def test_invalid_params_rejected(k, d, pl, msg):
    _ensure_built()
    lib = sdbg.load()
    p = sdbg._Params(k, d, 0, pl, 0, None)
    r = sdbg._Reads(None, None, 0, 0, 0)
    out = ctypes.POINTER(sdbg._Edges)()
    rc = lib.sdbg_count_solid(ctypes.byref(r), ctypes.byref(p), ctypes.byref(out))
    assert rc == -1
    assert msg in lib.sdbg_last_error().decode()
    assert not out


def test_null_arguments_rejected():
    _ensure_built()
    lib = sdbg.load()
    out = ctypes.POINTER(sdbg._Edges)()
    assert lib.sdbg_count_solid(None, None, ctypes.byref(out)) == -1
    g = ctypes.POINTER(sdbg._Graph)()
    assert lib.sdbg_build(None, None, ctypes.byref(g)) == -1
    # a pointer the library never returned is not an edge set
    fake = sdbg._Edges()
    assert lib.sdbg_build(ctypes.byref(fake), None, ctypes.byref(g)) == -1
    lib.sdbg_free(None)  # no-op


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(sdbg, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        sdbg.load(str(tmp_path / "nope.so"))


def test_tune_parameters_validated_on_host():
    """The launch-parameter setter is host-only: range checks and round trip."""
    _ensure_built()
    sdbg.load()
    sdbg.tune_set(None)
    default = sdbg.tune_get()
    assert default == {"digit_bits": 7, "tile_shift": 0, "leaf_wg_per_cu": 16, "leaf_cap_shift": 0, "first_bits": 6,
                       "mercy_shift": 0}
    for bad in ({"digit_bits": 3, "tile_shift": 0, "leaf_wg_per_cu": 16},
                {"digit_bits": 9, "tile_shift": 0, "leaf_wg_per_cu": 16},
                {"digit_bits": 8, "tile_shift": 2, "leaf_wg_per_cu": 16},
                {"digit_bits": 8, "tile_shift": 0, "leaf_wg_per_cu": 0},
                {"digit_bits": 8, "tile_shift": 0, "leaf_wg_per_cu": 33},
                {"digit_bits": 8, "tile_shift": 0, "leaf_wg_per_cu": 16, "leaf_cap_shift": 2},
                {"first_bits": 3}, {"first_bits": 9}, {"mercy_shift": 9}):
        with pytest.raises(sdbg.SdbgError) as ei:
            sdbg.tune_set(bad)
        assert ei.value.code == -1
        assert sdbg.tune_get() == default
    t = {"digit_bits": 6, "tile_shift": 1, "leaf_wg_per_cu": 8, "leaf_cap_shift": 1, "first_bits": 6,
         "mercy_shift": 3}
    sdbg.tune_set(t)
    assert sdbg.tune_get() == t
    sdbg.tune_set(None)
    assert sdbg.tune_get() == default


def test_graph_and_bwt_calls_reject_bad_arguments_on_the_host():
    """The unitig, cleaning, union, multi-k and BWT calls check their
    arguments before any device work: null pointers, objects the library
    never returned, and k values that do not ascend."""
    _ensure_built()
    sdbg.load()
    lib = ctypes.CDLL(sdbg.LIB_PATH)  # own function objects: the binding's signatures stay as they are
    lib.sdbg_last_error.restype = ctypes.c_char_p
    V = ctypes.c_void_p
    lib.sdbg_unitigs_build.argtypes = [V, V, V, V]
    lib.sdbg_merge_bubbles.argtypes = [V, V, V, ctypes.c_uint32, V, V]
    lib.sdbg_remove_low_coverage.argtypes = [V, V, V, ctypes.c_uint32, ctypes.c_uint32, V, V]
    lib.sdbg_remove_tips.argtypes = [V, V, ctypes.c_uint32, V, V]
    lib.sdbg_edges_union.argtypes = [V, V, V, V]
    lib.sdbg_multi_k.argtypes = [V, V, ctypes.c_uint32, V, V, V, V]
    lib.sdbg_read_bwt.argtypes = [V, V, V]
    lib.sdbg_bwt_to_host.argtypes = [V, V, V]
    lib.sdbg_unitigs_to_host.argtypes = [V, V, V, V, V, V]
    out = V()
    fake_g, fake_e = sdbg._Graph(), sdbg._Edges()
    gp, ep = ctypes.addressof(fake_g), ctypes.addressof(fake_e)
    assert lib.sdbg_unitigs_build(None, None, ctypes.byref(out), None) == -1
    assert lib.sdbg_unitigs_build(gp, gp, ctypes.byref(out), None) == -1  # not library objects
    assert lib.sdbg_merge_bubbles(gp, gp, gp, 10, None, None) == -1
    assert lib.sdbg_remove_low_coverage(gp, gp, gp, 10, 200, None, None) == -1
    assert lib.sdbg_remove_tips(gp, gp, 10, None, None) == -1
    assert lib.sdbg_edges_union(ep, ep, None, ctypes.byref(out)) == -1
    assert lib.sdbg_edges_union(None, ep, None, ctypes.byref(out)) == -1
    r = sdbg._Reads(None, None, 0, 0, 0)
    p = sdbg._Params(0, 2, 1, 8, 0, None)
    cl = sdbg._Clean(2, 2, 2, 200)
    ks = (ctypes.c_uint32 * 2)(41, 21)  # descending
    assert lib.sdbg_multi_k(ctypes.byref(r), ks, 2, ctypes.byref(p), ctypes.byref(cl), None, ctypes.byref(out)) == -1
    assert "ascend" in lib.sdbg_last_error().decode()
    ks_bad = (ctypes.c_uint32 * 1)(200)  # k out of range
    assert lib.sdbg_multi_k(ctypes.byref(r), ks_bad, 1, ctypes.byref(p), ctypes.byref(cl), None,
                            ctypes.byref(out)) == -1
    assert lib.sdbg_multi_k(ctypes.byref(r), ks, 2, ctypes.byref(p), None, None, ctypes.byref(out)) == -1
    assert lib.sdbg_read_bwt(None, None, ctypes.byref(out)) == -1
    assert lib.sdbg_bwt_to_host(gp, None, None) == -1
    assert lib.sdbg_unitigs_to_host(gp, None, None, None, None, None) == -1
    assert not out
