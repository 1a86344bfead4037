"""Seeded synthetic read sets shaped like the paper's workloads.

The paper assembles an E. coli MG1655 read set and an Iowa prairie soil
metagenome (Section 3, Tables 1-3).  Neither is available here, so every
input is simulated: random genomes, log-normal community abundances, reads
drawn uniformly from a genome on either strand, and iid substitution errors.
This module holds no part of the construction method (no k-mers, keys,
counting or graph logic); it is shared by the oracle tests, the device tests
and the benchmark.

Recipe (all draws from numpy's PCG64, seeded per workload):
  * genome bases iid uniform over A, C, G, T;
  * a community of G genomes has lengths log-uniform in [lo, hi]
    (exp of a uniform draw between ln lo and ln hi, rounded) and abundances
    exp(N(0, sigma^2)); a read comes from genome g with probability
    proportional to abundance_g * length_g;
  * a read of length L starts uniformly in [0, len_g - L] and is taken from
    the reverse-complement strand with probability 1/2;
  * each base is replaced, with probability p, by one of the other three
    bases chosen uniformly.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

MASTER_SEED = 0x14097208
_ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class ReadSet:
    """Reads as one ASCII byte string plus read boundaries.

    ``seq[offsets[i]:offsets[i+1]]`` is read i.  ``k``, ``d`` and ``mercy``
    are the construction parameters the workload is meant to be run with.
    """

    seq: np.ndarray  # uint8 ASCII, concatenated reads
    offsets: np.ndarray  # uint64, n_reads + 1
    k: int = 31
    d: int = 2
    mercy: bool = True
    name: str = ""

    @property
    def n_reads(self) -> int:
        return int(self.offsets.shape[0]) - 1

    def read(self, i: int) -> bytes:
        return self.seq[int(self.offsets[i]) : int(self.offsets[i + 1])].tobytes()

    def reads(self) -> list[bytes]:
        return [self.read(i) for i in range(self.n_reads)]

    def n_windows(self, k: int | None = None) -> int:
        """(k+1)-long windows over ACGT-only stretches, one strand."""
        k = self.k if k is None else k
        if self.seq.size == 0:
            return 0
        lengths = np.diff(self.offsets.astype(np.int64))
        bad = ~np.isin(self.seq, np.frombuffer(b"ACGTacgt", dtype=np.uint8))
        if not bad.any():
            return int(np.maximum(lengths - k, 0).sum())
        total = 0
        for r in self.reads():
            for seg in _split_acgt(r):
                total += max(0, len(seg) - k)
        return total

    def subset(self, n: int) -> "ReadSet":
        n = min(n, self.n_reads)
        end = int(self.offsets[n])
        return ReadSet(self.seq[:end].copy(), self.offsets[: n + 1].copy(), self.k, self.d, self.mercy, self.name + f"[:{n}]")


def _split_acgt(read: bytes) -> list[bytes]:
    out, cur = [], bytearray()
    for ch in read:
        if ch in b"ACGTacgt":
            cur.append(ch)
        else:
            if cur:
                out.append(bytes(cur))
            cur = bytearray()
    if cur:
        out.append(bytes(cur))
    return out


def rng_for(tag: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([MASTER_SEED ^ tag, extra]))


def random_genome(length: int, rng: np.random.Generator) -> np.ndarray:
    """Base codes 0..3 (A, C, G, T), iid uniform."""
    return rng.integers(0, 4, size=length, dtype=np.uint8)


def log_uniform_int(lo: float, hi: float, size, rng: np.random.Generator) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


@dataclasses.dataclass
class Community:
    genomes: np.ndarray  # uint8 codes, all genomes concatenated
    starts: np.ndarray  # int64, n_genomes + 1
    abundance: np.ndarray  # float64

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.starts)

    def read_weights(self) -> np.ndarray:
        w = self.abundance * self.lengths
        return w / w.sum()


def make_community(n_genomes: int, lo: int, hi: int, sigma: float, rng: np.random.Generator, log_uniform: bool = True) -> Community:
    if log_uniform:
        lengths = log_uniform_int(lo, hi, n_genomes, rng)
    else:
        lengths = rng.integers(lo, hi + 1, size=n_genomes).astype(np.int64)
    abundance = np.exp(rng.normal(0.0, sigma, size=n_genomes)) if sigma > 0 else np.ones(n_genomes)
    starts = np.zeros(n_genomes + 1, dtype=np.int64)
    np.cumsum(lengths, out=starts[1:])
    genomes = random_genome(int(starts[-1]), rng)
    return Community(genomes, starts, abundance)


def sample_reads(comm: Community, n_reads: int, read_len: int, err: float, rng: np.random.Generator, chunk: int = 1 << 18) -> tuple[np.ndarray, np.ndarray]:
    """Fixed-length reads; returns (ASCII bytes, offsets)."""
    L = int(read_len)
    lengths = comm.lengths
    if (lengths < L).any():
        raise ValueError("a genome is shorter than the read length")
    weights = comm.read_weights()
    seq = np.empty(n_reads * L, dtype=np.uint8)
    cols = np.arange(L, dtype=np.int64)
    done = 0
    while done < n_reads:
        c = min(chunk, n_reads - done)
        g = rng.choice(len(lengths), size=c, p=weights)
        start = (rng.random(c) * (lengths[g] - L + 1)).astype(np.int64)
        start = np.minimum(start, lengths[g] - L)
        rc = rng.integers(0, 2, size=c).astype(bool)
        idx = (comm.starts[g] + start)[:, None] + cols[None, :]
        codes = comm.genomes[idx]
        if rc.any():
            codes[rc] = 3 - codes[rc, ::-1]
        if err > 0:
            mask = rng.random((c, L), dtype=np.float32) < err
            nsub = int(mask.sum())
            if nsub:
                shift = rng.integers(1, 4, size=nsub, dtype=np.uint8)
                codes[mask] = (codes[mask] + shift) & 3
        seq[done * L : (done + c) * L] = _ASCII[codes].reshape(-1)
        done += c
    offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(L)
    return seq, offsets


# ---------------------------------------------------------------- workloads
# Index i is the workload's tag in the seed; sizes follow the five workloads
# the path is specified on.  ``scale`` shrinks read counts (and genome sizes
# for the community workloads) for quick tests while keeping the shape.

def tiny(scale: float = 1.0, seed_extra: int = 0) -> ReadSet:
    """50 kb random genome, 20,000 reads of 100 bp, 1% errors, k=21, d=2."""
    rng = rng_for(1, seed_extra)
    comm = make_community(1, 50_000, 50_000, 0.0, rng)
    n = max(1, int(round(20_000 * scale)))
    seq, off = sample_reads(comm, n, 100, 0.01, rng)
    return ReadSet(seq, off, k=21, d=2, mercy=False, name=f"tiny(scale={scale})")


_META_COMMUNITY_CACHE: dict = {}


def meta_community(scale: float = 1.0) -> Community:
    """200 genomes, log-uniform 1-5 Mb, log-normal abundance sigma=1.5.

    ``scale`` < 1 shrinks every genome length by that factor (keeping at
    least 1 kb) so that coverage per genome stays comparable in small tests.
    """
    key = scale
    if key in _META_COMMUNITY_CACHE:
        return _META_COMMUNITY_CACHE[key]
    rng = rng_for(2, 0)
    comm = make_community(200, 1_000_000, 5_000_000, 1.5, rng)
    if scale != 1.0:
        lengths = np.maximum((comm.lengths * scale).astype(np.int64), 1000)
        starts = np.zeros(len(lengths) + 1, dtype=np.int64)
        np.cumsum(lengths, out=starts[1:])
        genomes = np.concatenate([comm.genomes[comm.starts[i] : comm.starts[i] + lengths[i]] for i in range(len(lengths))])
        comm = Community(genomes, starts, comm.abundance)
    _META_COMMUNITY_CACHE.clear()
    _META_COMMUNITY_CACHE[key] = comm
    return comm


def metagenome(scale: float = 1.0, k: int = 31) -> ReadSet:
    """Community of 200 genomes, 10M reads of 100 bp, 0.5% errors, k=31, d=2, mercy on."""
    comm = meta_community(scale)
    rng = rng_for(2, 1)
    n = max(1, int(round(10_000_000 * scale)))
    seq, off = sample_reads(comm, n, 100, 0.005, rng)
    return ReadSet(seq, off, k=k, d=2, mercy=True, name=f"metagenome(scale={scale})")


def metagenome_long(scale: float = 1.0, k: int = 21) -> ReadSet:
    """Same community, 20M reads of 150 bp, 0.5% errors; k from 21, 41, 61, 81, 99."""
    comm = meta_community(scale)
    rng = rng_for(3, 1)
    n = max(1, int(round(20_000_000 * scale)))
    seq, off = sample_reads(comm, n, 150, 0.005, rng)
    return ReadSet(seq, off, k=k, d=2, mercy=True, name=f"metagenome_long(scale={scale},k={k})")


def batch_sets(n_sets: int = 4096, first: int = 0, read_scale: float = 1.0) -> list[ReadSet]:
    """Independent read sets, each from its own 20-500 kb genome (uniform),
    log-uniform 1k-1M reads of 100 bp, 1% errors, k=31, d=2."""
    meta = rng_for(4, 0)
    glen = meta.integers(20_000, 500_001, size=n_sets)
    nreads = log_uniform_int(1_000, 1_000_000, n_sets, meta)
    out = []
    for i in range(first, n_sets):
        rng = rng_for(4, 1 + i)
        comm = make_community(1, int(glen[i]), int(glen[i]), 0.0, rng, log_uniform=False)
        n = max(1, int(round(nreads[i] * read_scale)))
        seq, off = sample_reads(comm, n, 100, 0.01, rng)
        out.append(ReadSet(seq, off, k=31, d=2, mercy=False, name=f"batch[{i}]"))
    return out


def batch_set(i: int, n_sets: int = 4096, read_scale: float = 1.0) -> ReadSet:
    meta = rng_for(4, 0)
    glen = meta.integers(20_000, 500_001, size=n_sets)
    nreads = log_uniform_int(1_000, 1_000_000, n_sets, meta)
    rng = rng_for(4, 1 + i)
    comm = make_community(1, int(glen[i]), int(glen[i]), 0.0, rng, log_uniform=False)
    n = max(1, int(round(nreads[i] * read_scale)))
    seq, off = sample_reads(comm, n, 100, 0.01, rng)
    return ReadSet(seq, off, k=31, d=2, mercy=False, name=f"batch[{i}]")


def batch_set_device(i: int, n_sets: int = 4096, read_scale: float = 1.0, device: str = "cuda:0"):
    """Set i of the batch recipe drawn on the device with torch's generator
    (seeded per set): the same genome length, read count, read length,
    strand mix and error rate as batch_set(i), other random numbers.  For
    runs at full read scale, which are too large to draw on the host in a
    reasonable time (4096 sets hold about 590M reads).  Returns (ASCII reads,
    int64 offsets), both on the device."""
    import torch

    meta = rng_for(4, 0)
    glen = meta.integers(20_000, 500_001, size=n_sets)
    nreads = log_uniform_int(1_000, 1_000_000, n_sets, meta)
    seed = int(rng_for(4, 1 + i).integers(0, 2**62))
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    L, G = 100, int(glen[i])
    n = max(1, int(round(nreads[i] * read_scale)))
    genome = torch.randint(0, 4, (G,), generator=gen, device=device, dtype=torch.uint8)
    ascii = torch.tensor(list(b"ACGT"), dtype=torch.uint8, device=device)
    seq = torch.empty(n * L, dtype=torch.uint8, device=device)
    cols = torch.arange(L, device=device)
    for r0 in range(0, n, 1 << 18):
        c = min(1 << 18, n - r0)
        start = torch.randint(0, G - L + 1, (c,), generator=gen, device=device)
        codes = genome[start[:, None] + cols[None, :]]
        rc = torch.rand(c, generator=gen, device=device) < 0.5
        codes = torch.where(rc[:, None], 3 - codes.flip(1), codes)
        err = torch.rand((c, L), generator=gen, device=device) < 0.01
        shift = torch.randint(1, 4, (c, L), generator=gen, device=device, dtype=torch.uint8)
        codes = torch.where(err, (codes + shift) & 3, codes)
        seq[r0 * L : (r0 + c) * L] = ascii[codes.long()].reshape(-1)
    offsets = torch.arange(n + 1, device=device, dtype=torch.int64) * L
    return seq, offsets


@dataclasses.dataclass
class Job:
    arrival: float  # seconds from trace start
    reads: ReadSet


def serving_trace(rate: float, n_jobs: int, seed_extra: int = 0, read_scale: float = 1.0, genome_scale: float = 1.0) -> list[Job]:
    """Poisson arrivals of construction jobs: each job is a community of
    1-50 genomes (log-uniform 0.1-5 Mb, sigma=1.5), log-uniform 10k-20M reads
    of one length L uniform in [100, 150], 0.5% errors, k from {21, 41, 61}."""
    rng = rng_for(5, seed_extra)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    t = np.cumsum(gaps)
    jobs = []
    for j in range(n_jobs):
        jr, comm, n, L, k = _serving_job(j, seed_extra, read_scale, genome_scale)
        seq, off = sample_reads(comm, n, L, 0.005, jr)
        jobs.append(Job(float(t[j]), ReadSet(seq, off, k=k, d=2, mercy=True, name=f"job[{j}]")))
    return jobs


def _serving_job(j: int, seed_extra: int, read_scale: float, genome_scale: float):
    jr = rng_for(5, 1000 + seed_extra * 100_000 + j)
    ng = int(jr.integers(1, 51))
    comm = make_community(ng, max(200, int(100_000 * genome_scale)), max(400, int(5_000_000 * genome_scale)), 1.5, jr)
    n = max(1, int(round(float(log_uniform_int(10_000, 20_000_000, 1, jr)[0]) * read_scale)))
    L = int(jr.integers(100, 151))
    k = int(jr.choice([21, 41, 61]))
    return jr, comm, n, L, k


def serving_job_shapes(n_jobs: int, seed_extra: int = 0, read_scale: float = 1.0, genome_scale: float = 1.0) -> list[tuple[int, int, int]]:
    """(reads, read length, k) of the first n_jobs jobs of serving_trace,
    without sampling their reads."""
    return [_serving_job(j, seed_extra, read_scale, genome_scale)[2:] for j in range(n_jobs)]


def random_small(n_reads: int, min_len: int, max_len: int, genome_len: int, err: float, seed: int, n_rate: float = 0.0) -> ReadSet:
    """Small read sets for exhaustive checks: variable-length reads cut from a
    short random genome (so repeats and solid edges occur), optional 'N'
    bytes and lower-case bases."""
    rng = np.random.Generator(np.random.PCG64([MASTER_SEED, 77, seed]))
    genome = random_genome(max(genome_len, max_len), rng)
    parts, offs = [], [0]
    for _ in range(n_reads):
        L = int(rng.integers(min_len, max_len + 1))
        s = int(rng.integers(0, len(genome) - L + 1))
        codes = genome[s : s + L].copy()
        if rng.random() < 0.5:
            codes = 3 - codes[::-1]
        if err > 0:
            m = rng.random(L) < err
            codes[m] = (codes[m] + rng.integers(1, 4, size=int(m.sum()))) & 3
        b = _ASCII[codes].copy()
        if n_rate > 0:
            nm = rng.random(L) < n_rate
            b[nm] = ord("N")
            lower = rng.random(L) < 0.1
            b[lower & ~nm] = b[lower & ~nm] + 32
        parts.append(b)
        offs.append(offs[-1] + L)
    seq = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
    return ReadSet(seq, np.asarray(offs, dtype=np.uint64), name=f"random_small(seed={seed})")


def from_strings(reads: list[str], k: int, d: int = 2, mercy: bool = False) -> ReadSet:
    bs = [r.encode() for r in reads]
    offs = np.zeros(len(bs) + 1, dtype=np.uint64)
    np.cumsum([len(b) for b in bs], out=offs[1:])
    seq = np.frombuffer(b"".join(bs), dtype=np.uint8).copy()
    return ReadSet(seq, offs, k=k, d=d, mercy=mercy)
