"""Every HIP kernel of the library compiles for gfx950 without scratch
(private) memory: no register spills and no stack.  A kernel that needs
scratch makes the runtime allocate backing memory for its queue at
dispatch, which competes with the library's own device memory when several
jobs share the device.  Host-only: the check reads the compiler's resource
usage remarks."""

from __future__ import annotations

import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1409_7208_amd import build

CSRC = os.path.join(os.path.dirname(build.__file__), "csrc")
HIP_SOURCES = [s for s in build.SOURCES if s.endswith(".hip")]


def _resources(src: str) -> dict[str, dict[str, int]]:
    cmd = [build.hipcc(), *build._flags(), "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage", "-x", "hip",
           "-c", os.path.join(CSRC, src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out: dict[str, dict[str, int]] = {}
    cur = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if m and cur:
            out[cur][m.group(1).strip()] = int(m.group(2))
    return out


@pytest.fixture(scope="module")
def resources():
    with ThreadPoolExecutor(max_workers=len(HIP_SOURCES)) as ex:
        parts = list(ex.map(_resources, HIP_SOURCES))
    return {src: p for src, p in zip(HIP_SOURCES, parts)}


def test_kernels_found(resources):
    assert sum(len(v) for v in resources.values()) > 50
    assert any("k_leaf" in name for name in resources["count.hip"])


def test_no_kernel_uses_scratch(resources):
    # (SGPR spills go to VGPR lanes, not to scratch)
    bad = [(src, name, r.get("ScratchSize"), r.get("VGPRs Spill"))
           for src, kern in resources.items() for name, r in kern.items()
           if r.get("ScratchSize", 0) or r.get("VGPRs Spill", 0)]
    assert not bad, bad
