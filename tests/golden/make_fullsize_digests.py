"""Writes tests/golden/fullsize_digests.json: digests of the edge set and
SdBG arrays of each full-size workload, computed by the partitioned CPU
oracle (oracle.part_count_solid, oracle.part_build_graph) on the seeded
synthetic reads.  Calls nothing but oracle/ and the seeded generators.

    python tests/golden/make_fullsize_digests.py [workload ...]

workloads: metagenome (k = 31), long21, long41, long61, long81, long99.
Existing entries for other workloads are kept."""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import digests  # noqa: E402
import oracle  # noqa: E402
from paper_1409_7208_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")
ALL = ["metagenome", "long21", "long41", "long61", "long81", "long99"]


_LONG = {}


def reads_of(name: str):
    if name == "metagenome":
        return synth.metagenome(scale=1.0), 31
    k = int(name[4:])
    if "reads" not in _LONG:  # the same reads at every k
        _LONG["reads"] = synth.metagenome_long(scale=1.0)
    return _LONG["reads"], k


def main(names):
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    threads = min(16, os.cpu_count() or 1)
    for name in names:
        t0 = time.time()
        rs, k = reads_of(name)
        print(f"{name}: {rs.n_reads} reads generated in {time.time() - t0:.0f} s", flush=True)
        t1 = time.time()
        # groups of at most 2^29 keys keep the counting pass within ~16 GB
        e = oracle.part_count_solid(rs.seq, rs.offsets, k, 2, True, threads=threads, group_keys=1 << 29)
        t2 = time.time()
        print(f"  counted: {e.keys.shape[0]} edges ({e.n_mercy} mercy) of {e.n_occ} occurrences in {t2 - t1:.0f} s",
              flush=True)
        ed = digests.edge_digest(e.keys, e.counts, e.n_mercy, e.n_occ, k)
        g = oracle.part_build_graph(e.keys, e.counts, k, threads=threads)
        t3 = time.time()
        print(f"  built: m={g.m} t={g.t} in {t3 - t2:.0f} s", flush=True)
        table[name] = {"k": k, "d": 2, "mercy": True, "reads": rs.n_reads, "edges": ed,
                       "graph": digests.graph_digest(g), "oracle_seconds": round(t3 - t1, 1),
                       "oracle_threads": threads}
        del e, g
        with open(OUT, "w") as f:
            json.dump(table, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ALL)
