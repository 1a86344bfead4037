"""Host replays of device helpers (they are __host__ __device__), built
with hipcc for the host only and run on the CPU."""

from __future__ import annotations

import os
import subprocess

from paper_1409_7208_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


def test_rolling_window_packings(tmp_path):
    exe = str(tmp_path / "host_rolling")
    cmd = [build.hipcc(), "--cuda-host-only", "-O1", "-std=c++17", "-I", build.CSRC, "-x", "hip",
           os.path.join(HERE, "host_rolling.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
