"""Seeded synthetic inputs: random fully connected Ising instances and the
workload recipes measured by this package.

This module only draws random numbers and describes workloads; it holds none
of the annealing arithmetic, so both the GPU library's tests and the CPU
oracle can take their inputs from it.

The paper's instances (100 K8 and 100 K16 problems with J_ij uniform in
{+-0.1, ..., +-1} and h = 0, Sec. III) are not available; the stand-in is the
Sherrington-Kirkpatrick-like class J_ij uniform in {-1, +1}, h = 0, drawn from
numpy's PCG64 with a fixed seed per instance.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

ME = 0
LHZ = 1
MEC = 2          # ME on Chimera, chains of ceil(n/4)+1

SEED_SMALL = 1603          # the N=8 instance shared by the ME and LHZ single runs
SEED_BATCH = 20_000        # batched workload: instance i uses SEED_BATCH + i
SEED_PT = 30_000           # parallel-tempering workload: instance i uses SEED_PT + i
SEED_SERVE = 40_000        # serving job stream
ANNEAL_SEED_BASE = 0x5EED_0000_0000


def sk_instance(n: int, seed: int, values=(-1, 1)) -> np.ndarray:
    """J as an int32 n*n matrix, upper triangle drawn uniformly from `values`
    in row-major (i<j) order, zero elsewhere."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = np.zeros((n, n), dtype=np.int32)
    iu = np.triu_indices(n, 1)
    vals = np.asarray(values, dtype=np.int32)
    J[iu] = vals[rng.integers(0, len(vals), size=len(iu[0]))]
    return J


def n_sites(kind: int, n: int) -> int:
    """Physical spin count of the clique-chain ME (n(n-1)), LHZ (n(n-1)/2) and
    Chimera ME (n(ceil(n/4)+1)) layouts."""
    if kind == MEC:
        return n * ((n + 3) // 4 + 1)
    return n * (n - 1) if kind == ME else n * (n - 1) // 2


@dataclasses.dataclass
class AnnealJob:
    kind: int
    n: int
    J: np.ndarray
    penalty: int
    beta: float
    slices: int
    sweeps: int
    replicas: int
    gamma0: float
    gamma1: float
    seed: int

    @property
    def sites(self) -> int:
        return n_sites(self.kind, self.n)

    @property
    def attempts(self) -> int:
        return self.sites * self.slices * self.replicas * self.sweeps


def single_job(kind: int, sweeps: int = 1000, replicas: int = 16, slices: int = 32) -> AnnealJob:
    """The N=8 instance with ME (J_F = -2) or LHZ (C = -2): beta = 10,
    Gamma linear 3.0 -> 0.01."""
    return AnnealJob(kind, 8, sk_instance(8, SEED_SMALL), -2, 10.0, slices, sweeps, replicas,
                     3.0, 0.01, ANNEAL_SEED_BASE + kind)


def batch_jobs(count: int = 512, sweeps: int = 10_000, replicas: int = 64, slices: int = 64,
               sizes=(12, 16, 20, 24)) -> List[AnnealJob]:
    """Uneven batch: instance i is ME for even i, LHZ for odd i, with
    N = sizes[(i >> 1) % len(sizes)] (stratified, so every (N, embedding)
    pair appears equally often)."""
    jobs = []
    for i in range(count):
        kind = ME if i % 2 == 0 else LHZ
        n = sizes[(i >> 1) % len(sizes)]
        jobs.append(AnnealJob(kind, n, sk_instance(n, SEED_BATCH + i), -2, 10.0, slices, sweeps,
                              replicas, 3.0, 0.01, ANNEAL_SEED_BASE + 0x1000 + i))
    return jobs


@dataclasses.dataclass
class PTJob:
    kind: int
    n: int
    J: np.ndarray
    penalty: int
    temps: int
    beta_min: float
    beta_max: float
    sweeps: int
    sweeps_per_swap: int
    seed: int

    @property
    def sites(self) -> int:
        return n_sites(self.kind, self.n)


def pt_jobs(instances: int = 128, n: int = 24, temps: int = 32, sweeps: int = 100_000) -> List[PTJob]:
    """Every instance embedded both ways (LHZ and ME), 32 temperatures with beta
    geometric in [0.1, 5], a swap phase after every sweep."""
    jobs = []
    for i in range(instances):
        J = sk_instance(n, SEED_PT + i)
        for kind in (LHZ, ME):
            jobs.append(PTJob(kind, n, J, -2, temps, 0.1, 5.0, sweeps, 1,
                              ANNEAL_SEED_BASE + 0x100000 + 2 * i + kind))
    return jobs


def serving_stream(count: int, rate_per_s: float, seed: int = SEED_SERVE,
                   sweeps_range=(1000, 10_000), n_range=(8, 32), replicas: int = 16):
    """Poisson arrivals of anneal jobs: N uniform in n_range, embedding ME or LHZ
    at random, L in {32, 64}, sweeps uniform in sweeps_range.
    Returns a list of (arrival_time_s, AnnealJob)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        kind = int(rng.integers(0, 2))
        slices = 32 if rng.integers(0, 2) == 0 else 64
        sweeps = int(rng.integers(sweeps_range[0], sweeps_range[1] + 1))
        J = sk_instance(n, seed * 7919 + q)
        out.append((t, AnnealJob(kind, n, J, -2, 10.0, slices, sweeps, replicas, 3.0, 0.01,
                                 ANNEAL_SEED_BASE + 0x200000 + q)))
    return out
