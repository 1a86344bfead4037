"""Host replays of device helpers (they are __host__ __device__), built
with hipcc for the host only, with the undefined-behaviour sanitizer, and
run on the CPU."""

from __future__ import annotations

import os
import subprocess

from paper_1409_7208_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
# sanitizer flags for the host pass only (these builds have no device pass)
UBSAN = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(tmp_path, src: str) -> None:
    exe = str(tmp_path / os.path.splitext(src)[0])
    cmd = [build.hipcc(), "--cuda-host-only", "-O1", "-g", "-std=c++17", *UBSAN, "-I", build.CSRC, "-x", "hip",
           os.path.join(HERE, src), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_rolling_window_packings(tmp_path):
    """Rolling forward/reverse-complement packings equal the packings built
    from the stream, every key width, k = 2..127."""
    _run(tmp_path, "host_rolling.cpp")


def test_word_slot_table_replay(tmp_path):
    """The word-slot mercy table (keys of 2-4 words): fill by every solid
    key, lookups with 1, 2 and 4 windows per thread, overfull buckets
    included, equal a binary search of the sorted set, with no undefined
    behaviour on the way."""
    _run(tmp_path, "host_wslot.cpp")
