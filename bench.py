"""Throughput of SdBG construction (count + solid filter + mercy + SdBG
arrays) on one MI355X.

One step = sdbg_count_solid + sdbg_build over the whole read set, reads
already resident in HBM, outputs left in HBM.  Prints one JSON line.

Workload (default): a synthetic metagenome shaped like the paper's soil
data set (Section 3): 200 random genomes of log-uniform 1-5 Mb with
log-normal abundances (sigma 1.5), 10M reads of 100 bp at 0.5% substitution
errors, k=31, d=2, mercy-kmers on.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gmer/s sort+count+SdBG build (frac of HBM roofline); p99 job latency vs plain"
HBM_PEAK_GBS = 8000.0


# HBM traffic of the dominant kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counter runs scaled by a 1 GiB device copy (profiles/), valid
# while the kernel sources hash to the value recorded there.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_metagenome_k31.md")
KERNEL_SOURCES = ["paper_1409_7208_amd/csrc/" + f for f in
                  ("count.hip", "build.hip", "prims.hip", "device.h", "kernels.h", "prims.h", "windows.h", "wslots.h")]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(stage: str, workload: str):
    """Bytes per launch recorded for `stage` on the headline workload, or None."""
    if workload != "metagenome" or not os.path.exists(TRAFFIC_FILE):
        return None
    src = kernel_source_hash()
    for line in open(TRAFFIC_FILE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 3 and cells[0] == stage and cells[-1] == src:
            try:
                return float(cells[-2])
            except ValueError:
                return None
    return None


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name: str, scale: float):
    from paper_1409_7208_amd import synth

    if name == "metagenome":
        rs = synth.metagenome(scale=scale)
        desc = "metagenome: 200 genomes log-uniform 1-5 Mb, log-normal abundance sigma 1.5, 10M reads x 100 bp, 0.5% err, k=31, d=2, mercy"
    elif name == "tiny":
        rs = synth.tiny(scale=scale)
        desc = "tiny: 50 kb genome, 20k reads x 100 bp, 1% err, k=21, d=2"
    elif name.startswith("long"):
        k = int(name[4:] or 21)
        rs = synth.metagenome_long(scale=scale, k=k)
        desc = f"metagenome long reads: 20M reads x 150 bp, k={k}, d=2, mercy"
    else:
        raise SystemExit(f"unknown workload {name}")
    if scale != 1.0:
        desc += f" (scale {scale})"
    return rs, desc


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rs, n_reads: int, n_reads_single: int):
    """The oracle as it stands, on the host cores: the partitioned oracle
    (the same definitions block by block on a thread pool, the CPU
    counterpart of the construction) on the first n_reads reads, and the
    string oracle on one thread on the first n_reads_single reads."""
    import oracle

    threads = min(16, os.cpu_count() or 1)
    sub = rs.subset(n_reads)
    t0 = time.perf_counter()
    e = oracle.part_count_solid(sub.seq, sub.offsets, rs.k, rs.d, rs.mercy, threads=threads)
    oracle.part_build_graph(e.keys, e.counts, rs.k, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": e.n_occ / dt / 1e9, "unit": "Gmer/s", "cores": threads, "kind": "oracle",
           "sample": f"first {sub.n_reads} reads of the workload ({e.n_occ} (k+1)-mer occurrences), count+build by "
                     f"the partitioned oracle (256 key blocks on {threads} threads), {dt:.1f} s",
           "cpu_model": cpu_model()}
    sub1 = rs.subset(n_reads_single)
    t0 = time.perf_counter()
    e1 = oracle.count_solid(sub1.seq, sub1.offsets, rs.k, rs.d, rs.mercy)
    oracle.build_graph(e1.keys, e1.counts, rs.k)
    dt1 = time.perf_counter() - t0
    out["single_thread"] = {"value": e1.n_occ / dt1 / 1e9, "unit": "Gmer/s", "cores": 1,
                            "sample": f"first {sub1.n_reads} reads, string oracle, {dt1:.1f} s"}
    return out


def large_k_rates(steps: int):
    """Gmer/s of the large-k workload (same community, 20M reads x 150 bp,
    mercy on) at each k, reads resident on the device; HBM traffic per
    occurrence from the library's per-launch algorithmic bytes."""
    import torch

    from paper_1409_7208_amd import sdbg, synth

    t0 = time.perf_counter()
    rs = synth.metagenome_long()
    log(f"large-k workload: {rs.n_reads} reads generated in {time.perf_counter() - t0:.1f} s")
    seq = torch.from_numpy(rs.seq).to("cuda:0")
    off = torch.from_numpy(rs.offsets.view(np.int64)).to("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for k in (21, 41, 61, 81, 99):
        def step():
            e = sdbg.count_solid(seq, off, k, 2, True, stream=stream)
            g = sdbg.build(e, stream=stream)
            res = (e.n_occ, e.n)
            g.close()
            e.close()
            return res

        step()
        torch.cuda.synchronize()
        sdbg.profile_enable(True)
        sdbg.profile_reset()
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        for _ in range(steps):
            r = step()
        eb.record(stream)
        torch.cuda.synchronize()
        sdbg.profile_enable(False)
        ms = ea.elapsed_time(eb) / steps
        step_bytes = sum(b for _, _, b in sdbg.profile_records()) / steps
        gms = r[0] / (ms / 1e3) / 1e9
        rows.append({"k": k, "n_occ": int(r[0]), "edges": int(r[1]), "ms_per_step": round(ms, 2),
                     "gmer_s": round(gms, 3), "bytes_per_occ": round(step_bytes / r[0], 1),
                     "step_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        log(f"large k={k}: {ms:.1f} ms/step, {gms:.2f} Gmer/s")
    multi = multi_k_run(sdbg, torch, seq, off, stream)
    del seq, off
    torch.cuda.synchronize()
    return rows, multi


def multi_k_run(sdbg, torch, seq, off, stream, ks=(21, 41, 61, 81, 99)):
    """One pass of the multi-k workflow over the large-k workload: per k the
    reads' solid edges (mercy on) united with the previous k's unitigs,
    graph, tips, bubbles and low-coverage unitigs of at most 2k edges
    removed (ratio 0.2), unitigs (HIP events)."""
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ea.record(stream)
    u, st = sdbg.multi_k(seq, off, list(ks), d=2, mercy=True, tip_factor=2, bubble_factor=2, low_cov_factor=2,
                         low_cov_permille=200, stream=stream)
    eb.record(stream)
    torch.cuda.synchronize()
    ms = ea.elapsed_time(eb)
    out = {"ks": list(ks), "ms": round(ms, 1), "unitigs": int(u.n), "bases": int(u.n_bases),
           "clean": {"tip_factor": 2, "bubble_factor": 2, "low_cov_factor": 2, "low_cov_permille": 200},
           "per_k": [{"k": k, "edges": int(a), "from_unitigs": int(b), "tip_edges": int(c), "bubble_edges": int(d),
                      "low_cov_edges": int(e), "unitigs": int(f)} for k, (a, b, c, d, e, f) in zip(ks, st.tolist())]}
    u.close()
    log(f"multi-k {list(ks)}: {ms:.0f} ms, {out['unitigs']} unitigs at k={ks[-1]}; per k {st.tolist()}")
    return out


def navigation_rates(sdbg, torch, seq, off, rs, stream):
    """Navigation index build, tip removal (paths of at most 2k edges),
    unitigs of the cleaned graph and random forward queries on one graph of
    the workload, outside the timed steps (HIP events on the call stream)."""
    e = sdbg.count_solid(seq, off, rs.k, rs.d, rs.mercy, stream=stream)
    g = sdbg.build(e, stream=stream)
    e.close()
    torch.cuda.synchronize()
    ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    ea.record(stream)
    ix = sdbg.Index(g, stream=stream)
    eb.record(stream)
    removed = ix.remove_tips(2 * rs.k, stream=stream)
    ec.record(stream)
    torch.cuda.synchronize()
    eu0, eu1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    eu0.record(stream)
    u = ix.unitigs(stream=stream)
    eu1.record(stream)
    torch.cuda.synchronize()
    hl = u.to_host()
    unitigs = {"unitigs_ms": round(eu0.elapsed_time(eu1), 3), "unitigs": int(u.n), "cycles": int(u.n_cycles),
               "bases": int(u.n_bases), "longest_edges": int(hl.len.max()) if u.n else 0}
    u.close()
    del hl
    rows = torch.randint(0, int(g.raw.m), (1 << 24,), device="cuda:0", dtype=torch.int64)
    outq = torch.empty_like(rows)
    ed, ee = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ix.navigate(sdbg.NAV_FORWARD, rows, outq, stream=stream)
    ed.record(stream)
    ix.navigate(sdbg.NAV_FORWARD, rows, outq, stream=stream)
    ee.record(stream)
    torch.cuda.synchronize()
    clean = {"index_ms": round(ea.elapsed_time(eb), 3), "remove_tips_ms": round(eb.elapsed_time(ec), 3),
             "tip_max_len": 2 * rs.k, "tip_edges_removed": int(removed),
             "forward_queries_per_s": round((1 << 24) / (ed.elapsed_time(ee) * 1e-3), 1), **unitigs}
    log(f"index {clean['index_ms']} ms, tip removal {clean['remove_tips_ms']} ms ({removed} edges), "
        f"unitigs {unitigs['unitigs_ms']} ms ({unitigs['unitigs']}, longest {unitigs['longest_edges']} edges), "
        f"{clean['forward_queries_per_s'] / 1e9:.2f} G forward queries/s")
    ix.close()
    g.close()
    del rows, outq
    return clean


def bwt_rate(sdbg, torch, seq, off, stream):
    """The read-set BWT (every suffix of the workload's reads sorted, on the
    device; the result is not copied back), HIP events on the call stream."""
    sdbg.read_bwt(seq, off, stream=stream, to_host=False)  # warm-up
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ea.record(stream)
    n = sdbg.read_bwt(seq, off, stream=stream, to_host=False)
    eb.record(stream)
    torch.cuda.synchronize()
    ms = ea.elapsed_time(eb)
    out = {"suffixes": int(n), "ms": round(ms, 1), "suffixes_per_s": round(n / (ms * 1e-3), 1)}
    log(f"read BWT: {n} suffixes in {ms:.0f} ms ({out['suffixes_per_s'] / 1e9:.2f} G suffixes/s)")
    return out


def bench_batch(args):
    """Batched form against one plain call per set, on the same device-resident
    sets; both build the SdBG of every set."""
    import torch

    from paper_1409_7208_amd import sdbg, synth

    sdbg.load()
    torch.cuda.set_device(0)
    scale = 0.01 if args.read_scale is None else args.read_scale
    t0 = time.perf_counter()
    if args.gen_device:
        dev = [synth.batch_set_device(i, read_scale=scale) for i in range(args.sets)]
        n_reads = sum(int(o.numel()) - 1 for _, o in dev)
    else:
        sets = [synth.batch_set(i, read_scale=scale) for i in range(args.sets)]
        n_reads = sum(r.n_reads for r in sets)
        dev = [(torch.from_numpy(r.seq).to("cuda:0"), torch.from_numpy(r.offsets.view(np.int64)).to("cuda:0"))
               for r in sets]
        del sets
    torch.cuda.synchronize()
    log(f"generated {len(dev)} sets, {n_reads} reads in {time.perf_counter() - t0:.1f} s"
        f"{' (on the device)' if args.gen_device else ''}")
    stream = torch.cuda.current_stream()

    def batched():
        res = sdbg.batch_run(dev, 31, 2, False, stream=stream)
        occ = sum(e.n_occ for e, _ in res)
        for e, g in res:
            e.close()
            g.close()
        return occ

    def sequential():
        occ = 0
        for seq, off in dev:
            e = sdbg.count_solid(seq, off, 31, 2, False, stream=stream)
            g = sdbg.build(e, stream=stream)
            occ += e.n_occ
            g.close()
            e.close()
        return occ

    tuned = None
    if args.autotune:
        # tune on every 16th set (a sample of the size mix), then time all
        sample = dev[::16]
        t0 = time.perf_counter()
        tuned = sdbg.autotune(sample, 31, reps=1)
        log(f"autotune on {len(sample)} sets picked {tuned} in {time.perf_counter() - t0:.1f} s")
    out = {}
    for name, fn in (("batched", batched), ("sequential", sequential)):
        fn()  # warm-up (device memory pool)
        torch.cuda.synchronize()
        times = []
        if args.stages:
            sdbg.profile_enable(True)
            sdbg.profile_reset()
        for _ in range(max(1, args.steps)):
            w0 = time.perf_counter()
            occ = fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - w0)
        if args.stages:
            sdbg.profile_enable(False)
            agg: dict[str, list] = {}
            for kname, kt, kb in sdbg.profile_records():
                a = agg.setdefault(kname, [0, 0.0, 0])
                a[0] += 1
                a[1] += kt
                a[2] += kb
            steps = max(1, args.steps)
            for kname, (n, kt, kb) in sorted(agg.items(), key=lambda x: -x[1][1])[:14]:
                log(f"  {name} {kname:14s} launches={n // steps:6d}  {kt / steps:9.2f} ms  "
                    f"{kb / (kt * 1e-3) / 1e9 if kt > 0 else 0:8.1f} GB/s")
        t = float(np.median(times))
        out[name] = {"seconds": round(t, 4), "gmer_s": round(occ / t / 1e9, 3)}
        log(f"{name}: {t * 1e3:.1f} ms, {occ / t / 1e9:.3f} Gmer/s over {len(dev)} sets")
    line = {"metric": "Gmer/s batched form vs one call per set", "form": "batch", "value": out["batched"]["gmer_s"],
            "unit": "Gmer/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"first {len(dev)} sets of 4096: genome 20-500 kb, log-uniform 1k-1M reads "
                                   f"x {scale} of 100 bp, 1% err, k=31, d=2, mercy off", "reads": n_reads,
                       "n_occ": int(occ), "generator": "device" if args.gen_device else "host"},
            "batched": out["batched"], "sequential": out["sequential"], "tune": tuned or sdbg.tune_get(),
            "speedup": round(out["sequential"]["seconds"] / out["batched"]["seconds"], 3)}
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """Poisson request stream through the request loop (4 jobs at once)
    against the same trace run one job at a time; latency = submit to
    completion of the job's SdBG arrays."""
    import threading

    import torch

    from paper_1409_7208_amd import sdbg, synth

    sdbg.load()
    torch.cuda.set_device(0)
    scale = 0.5 if args.read_scale is None else args.read_scale
    t0 = time.perf_counter()
    pool = [j.reads for j in synth.serving_trace(1.0, args.pool, read_scale=scale, genome_scale=0.1)]
    log(f"generated {len(pool)} jobs, {sum(r.n_reads for r in pool)} reads in {time.perf_counter() - t0:.1f} s")

    def replay(max_jobs, arrivals, jobs):
        """One replay of the trace; every wait is bounded by a deadline, on
        whose expiry the request loop's state is printed and the run ends."""
        res = [None] * len(jobs)
        deadline = time.perf_counter() + args.serve_deadline
        with sdbg.Server(max_jobs=max_jobs) as srv:
            ids = [None] * len(jobs)
            failed = []

            def submitter():
                base = time.perf_counter()
                try:
                    for i, (a, rs) in enumerate(zip(arrivals, jobs)):
                        dt = base + a - time.perf_counter()
                        if dt > 0:
                            time.sleep(dt)
                        ids[i] = srv.submit(rs.seq, rs.offsets, rs.k, 2, True)
                except Exception as e:  # reported by the main thread
                    failed.append(e)

            def stuck(what):
                st = srv.state()
                log(f"serve replay ({max_jobs} jobs at once) stuck {what}: {st}")
                for i, jid in enumerate(ids):
                    if jid is not None and res[i] is None:
                        tr = srv.trace(jid)
                        r = srv.poll(jid, wait=False)
                        log(f"  job {i} (id {jid}, k={jobs[i].k}, {jobs[i].n_reads} reads): status {r.status}, "
                            f"submit {r.submit_s:.3f} s start {r.start_s:.3f} s footprint {r.footprint}, "
                            f"at {tr}")
                sys.stderr.flush()
                os._exit(3)

            th = threading.Thread(target=submitter, daemon=True)
            th.start()
            for i in range(len(jobs)):
                while ids[i] is None:
                    if failed:
                        raise failed[0]
                    if time.perf_counter() > deadline:
                        stuck(f"waiting for submission of job {i}")
                    time.sleep(0.002)
                while True:
                    r = srv.poll(ids[i], wait=False)
                    if r.status <= 0:
                        break
                    if time.perf_counter() > deadline:
                        stuck(f"waiting for job {i}")
                    time.sleep(0.002)
                assert r.status == 0, r.error
                res[i] = (r.submit_s, r.start_s, r.end_s, r.n_occ)
                r.edges.close()
                r.graph.close()
            th.join()
        lat = np.array([e - s for s, _, e, _ in res])
        span = max(e for _, _, e, _ in res) - min(s for s, _, _, _ in res)
        occ = sum(o for *_, o in res)
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "gmer_s": round(occ / span / 1e9, 3), "jobs": len(jobs), "n_occ": int(occ)}

    # warm the device memory pool on the largest job
    big = max(pool, key=lambda r: r.n_reads)
    replay(1, [0.0], [big])
    rng = np.random.default_rng(0x14097208)
    rows = []
    for lam in [float(x) for x in args.rates.split(",")]:
        n = int(min(len(pool), max(8, 4 * lam)))
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n))
        arrivals -= arrivals[0]
        jobs = [pool[i % len(pool)] for i in range(n)]
        cb = replay(4, arrivals, jobs)
        fifo = replay(1, arrivals, jobs)
        rows.append({"rate": lam, "served": cb, "one_at_a_time": fifo})
        log(f"rate {lam:5.1f}/s: served p50 {cb['p50_ms']} ms p99 {cb['p99_ms']} ms {cb['gmer_s']} Gmer/s | "
            f"one-at-a-time p50 {fifo['p50_ms']} ms p99 {fifo['p99_ms']} ms {fifo['gmer_s']} Gmer/s")
    top = rows[-1]
    line = {"metric": "p99 job latency and aggregate Gmer/s, request loop vs one job at a time", "form": "serve",
            "value": top["served"]["gmer_s"], "unit": "Gmer/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"Poisson jobs: 1-50 genomes of 0.01-0.5 Mb, log-uniform 10k-20M reads x {scale}, "
                                   "L 100-150, 0.5% err, k in {21,41,61}, d=2, mercy", "pool": len(pool),
                       "max_jobs": 4},
            "rates": rows}
    print(json.dumps(line), flush=True)


def parse_tune(spec: str) -> dict:
    t = {}
    for part in spec.split(","):
        if part.strip():
            k, v = part.split("=")
            t[k.strip()] = int(v)
    return t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="metagenome")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--cpu-reads", type=int, default=1000000, help="reads of the partitioned-oracle CPU baseline")
    ap.add_argument("--cpu-reads-single", type=int, default=50000, help="reads of the single-thread oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large-k", action="store_true", help="skip the large-k figures (k = 21..99)")
    ap.add_argument("--large-k-steps", type=int, default=2)
    ap.add_argument("--no-nav", action="store_true", help="skip the navigation, cleaning, unitig and read-BWT figures")
    ap.add_argument("--stages", action="store_true", help="print per-kernel breakdown to stderr")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (a reference kernel for hardware byte counters)")
    ap.add_argument("--form", default="plain", choices=["plain", "batch", "serve"],
                    help="plain: one job (the headline); batch: many read sets per call vs one call per set; "
                         "serve: Poisson request stream through the request loop vs one job at a time")
    ap.add_argument("--sets", type=int, default=4096, help="batch: first N sets of the 4096-set recipe")
    ap.add_argument("--gen-device", action="store_true", help="batch: draw the sets on the device (full read scale)")
    ap.add_argument("--read-scale", type=float, default=None, help="batch/serve: scale of the read counts")
    ap.add_argument("--rates", default="1,2", help="serve: arrival rates (jobs/s); see the design notes before "
                    "running 5 and above")
    ap.add_argument("--pool", type=int, default=32, help="serve: distinct jobs in the pool")
    ap.add_argument("--serve-deadline", type=float, default=120.0,
                    help="serve: seconds one replay may take before the loop's state is printed and the run ends")
    ap.add_argument("--autotune", action="store_true", help="batch: pick launch parameters on a sample first")
    ap.add_argument("--tune", default="", help="launch parameters, e.g. leaf_cap_shift=1,leaf_wg_per_cu=8")
    ap.add_argument("--host-input", action="store_true",
                    help="plain: also time a step that takes the reads from host memory (PCIe included), stderr only")
    ap.add_argument("--sweep", default="",
                    help="plain: also time these launch-parameter settings (';'-separated --tune strings), stderr only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.form == "batch":
        return bench_batch(args)
    if args.form == "serve":
        return bench_serve(args)

    import torch

    from paper_1409_7208_amd import sdbg

    sdbg.load()
    torch.cuda.set_device(0)
    if args.tune:
        sdbg.tune_set(parse_tune(args.tune))
    t0 = time.perf_counter()
    rs, desc = make_workload(args.workload, args.scale)
    log(f"generated {rs.n_reads} reads in {time.perf_counter() - t0:.1f} s")
    seq = torch.from_numpy(rs.seq).to("cuda:0")
    off = torch.from_numpy(rs.offsets.view(np.int64)).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.int64, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        e = sdbg.count_solid(seq, off, rs.k, rs.d, rs.mercy, stream=stream)
        g = sdbg.build(e, stream=stream)
        res = (e.n_occ, e.n, e.n_mercy, g.m, g.t)
        g.close()
        e.close()
        return res

    for i in range(args.warmup):
        r = step()
        log(f"warmup {i}: n_occ={r[0]} edges={r[1]} mercy={r[2]} m={r[3]} t={r[4]}")
    torch.cuda.synchronize()
    sdbg.profile_enable(True)
    sdbg.profile_reset()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        r = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    sdbg.profile_enable(False)
    ms = ev0.elapsed_time(ev1) / args.steps
    n_occ = r[0]
    value = n_occ / (ms / 1e3) / 1e9
    log(f"timed {args.steps} steps: {ms:.2f} ms/step (wall {wall / args.steps * 1e3:.2f} ms/step), {value:.2f} Gmer/s")

    for spec in [x for x in args.sweep.split(";") if x.strip()]:
        base = sdbg.tune_get()
        sdbg.tune_set(parse_tune(spec))
        step()
        torch.cuda.synchronize()
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        for _ in range(args.steps):
            step()
        eb.record(stream)
        torch.cuda.synchronize()
        sms = ea.elapsed_time(eb) / args.steps
        log(f"sweep {spec}: {sms:.2f} ms/step, {n_occ / (sms / 1e3) / 1e9:.2f} Gmer/s")
        sdbg.tune_set(base)

    host_rate = None
    if args.host_input:
        seq_h, off_h = rs.seq, rs.offsets
        e = sdbg.count_solid(seq_h, off_h, rs.k, rs.d, rs.mercy, stream=stream)
        sdbg.build(e, stream=stream).close()
        e.close()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(args.steps):
            e = sdbg.count_solid(seq_h, off_h, rs.k, rs.d, rs.mercy, stream=stream)
            sdbg.build(e, stream=stream).close()
            e.close()
        torch.cuda.synchronize()
        hms = (time.perf_counter() - w0) / args.steps * 1e3
        host_rate = n_occ / (hms / 1e3) / 1e9
        log(f"host input (PCIe copy of reads included): {hms:.2f} ms/step, {host_rate:.2f} Gmer/s")

    recs = sdbg.profile_records()
    if args.stages:
        per_step = len(recs) // args.steps
        log("  launches of the last step (ms, GB/s):")
        for name, t, b in recs[-per_step:]:
            log(f"    {name:14s} {t:9.3f} {b / (t * 1e-3) / 1e9 if t > 0 else 0:9.1f}")
    agg: dict[str, list] = {}
    for name, t, b in recs:
        a = agg.setdefault(name, [0, 0.0, 0])
        a[0] += 1
        a[1] += t
        a[2] += b
    total_prof = sum(a[1] for a in agg.values())
    if args.stages or True:
        for name, (n, t, b) in sorted(agg.items(), key=lambda x: -x[1][1]):
            log(f"  {name:14s} launches={n // args.steps:3d}/step  {t / args.steps:8.3f} ms/step  "
                f"{b / (t * 1e-3) / 1e9 if t > 0 else 0:8.1f} GB/s  ({100 * t / args.steps / ms:5.1f}% of step)")
        log(f"  profiled kernels cover {100 * total_prof / args.steps / ms:.1f}% of the step")
    dom = max(agg.items(), key=lambda x: x[1][1])
    dn, (dcnt, dms, dbytes) = dom
    achieved = dbytes / (dms * 1e-3) / 1e9
    traffic = recorded_traffic(dn, args.workload) if args.scale == 1.0 else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dn,
                "avg_launch_ms": round(dms / dcnt, 4), "bytes_per_launch": int(dbytes / dcnt)}

    # Whole step against the HBM roofline: every profiled launch's algorithmic
    # bytes over the step time, and the floor of a one-partition-pass
    # schedule (32 w bytes per occurrence for extraction write, one
    # partition pass and the leaf read, plus 8w+4 per output edge).
    w = (2 * (rs.k + 1) + 63) // 64
    step_bytes = sum(a[2] for a in agg.values()) / args.steps
    floor_b = 32 * w + (int(r[1]) / n_occ) * (8 * w + 4)
    step_roofline = {"bytes_per_occ": round(step_bytes / n_occ, 2),
                     "achieved_gbs": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                     "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "floor_bytes_per_occ": round(floor_b, 2),
                     "floor_frac": round(value * floor_b / HBM_PEAK_GBS, 4)}

    clean = bwt = None
    if not args.no_nav:
        clean = navigation_rates(sdbg, torch, seq, off, rs, stream)
        try:
            bwt = bwt_rate(sdbg, torch, seq, off, stream)
        except sdbg.SdbgError as e:  # reads with non-base bytes have no BWT here
            bwt = {"error": str(e)}

    large = multi = None
    if not args.no_large_k and args.workload == "metagenome" and args.scale == 1.0:
        del seq, off
        large, multi = large_k_rates(args.large_k_steps)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(rs, args.cpu_reads, args.cpu_reads_single)
        log(f"  {cpu}")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gmer/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "k": rs.k, "d": rs.d, "mercy": rs.mercy, "reads": rs.n_reads,
                   "n_occ": int(n_occ), "edges": int(r[1]), "mercy_edges": int(r[2]), "rows": int(r[3]),
                   "tips": int(r[4])},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_roofline": step_roofline,
        "tune": sdbg.tune_get(),
    }
    if host_rate is not None:
        out["host_input_gmer_s"] = round(host_rate, 3)
    if large is not None:
        out["large_k"] = large
        out["multi_k"] = multi
    if clean is not None:
        out["navigation"] = clean
        out["read_bwt"] = bwt
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
