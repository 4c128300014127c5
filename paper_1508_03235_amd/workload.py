"""Seeded synthetic workload inputs: model parameters and Zipf quantile tables.

This module generates inputs only; it holds none of the simulator's arithmetic and is
the one module both the HIP path and the serial oracle take their inputs from.

The paper drives its simulator with per-core address traces recorded with Multi2sim
(Sec. 6.2.3, trace generation).  Those traces are not available, so every core draws
its own address stream: a per-cycle Bernoulli coin issues a memory operation, a second
coin picks the shared or the tile's private region, and a Zipf-distributed rank picks
the line inside the region.  The rank comes from a quantile table built here once in
float64: entry b is the smallest rank whose cumulative probability exceeds b/K, and
entry K is the region size.  Both sides receive the same table as data.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field, replace, asdict

import numpy as np

ZIPF_K = 65536

# model-parameter field order shared by every consumer of a config dict
FIELDS = (
    "width", "height", "seed", "l1_sets", "l1_ways", "l2_sets", "l2_ways", "l1_lat",
    "mem_lat", "op_thr", "shared_thr", "bg_thr", "shared_lines", "private_lines",
    "zipf_shared_s", "zipf_private_s", "reply_flits", "flags", "router_delay", "mig_threshold",
)

# Model variants (bits of SimParams.flags), each a more literal reading of one passage of the
# paper than the base model's: priority by deflection count (AGE_DEFLECT), a core that keeps
# serving hits while its miss is outstanding (HIT_UNDER_MISS), and a flit entering the network
# the cycle after it is made (INJECT_DELAY).
AGE_DEFLECT = 1
HIT_UNDER_MISS = 2
INJECT_DELAY = 4
# The paper's logically shared, physically distributed L2 with a directory (local placement,
# directory access / reply, remote access, traps, eviction notices); the directory is
# interleaved over the tiles by line, or with LSPD_CENTRAL kept by the tile at the mesh centre.
LSPD = 8
LSPD_CENTRAL = 16


def thr(p: float) -> int:
    """Bernoulli threshold for probability p: a uniform u32 draw u succeeds iff u < thr."""
    if p <= 0.0:
        return 0
    return min(int(math.floor(p * 2.0**32)), 2**32 - 1)


@functools.lru_cache(maxsize=8)
def zipf_table(n: int, s: float, k: int = ZIPF_K) -> np.ndarray:
    """Quantile table (k+1 uint32 entries) of P(rank = j) proportional to (j+1)^-s, j < n."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    b = np.arange(k, dtype=np.float64) / k
    q = np.empty(k + 1, dtype=np.uint32)
    q[:k] = np.minimum(np.searchsorted(cdf, b, side="right"), n - 1)
    q[k] = n
    q.setflags(write=False)
    return q


@dataclass(frozen=True)
class SimParams:
    """One simulated chip: mesh shape, seed, cache shapes, latencies and traffic rates."""
    width: int
    height: int
    seed: int
    l1_sets: int = 128        # 32 KB, 4-way, 64 B lines
    l1_ways: int = 4
    l2_sets: int = 512        # 256 KB, 8-way, 64 B lines per tile
    l2_ways: int = 8
    l1_lat: int = 1
    mem_lat: int = 200
    op_thr: int = 2**30       # one memory op per 4 cycles
    shared_thr: int = 2**32 - 1
    bg_thr: int = 0
    shared_lines: int = 2**20
    private_lines: int = 0
    zipf_shared_s: float = 0.8
    zipf_private_s: float = 0.9
    reply_flits: int = 1      # flits per reply packet (the paper's Table 1: 4 for a remote L2 access)
    flags: int = 0            # model variants: AGE_DEFLECT | HIT_UNDER_MISS | INJECT_DELAY | LSPD [| LSPD_CENTRAL]
    router_delay: int = 1     # cycles per hop (a flit waits router_delay - 1 cycles in each router)
    mig_threshold: int = 0    # LSPD: history length N (<= 16); a block migrates to a tile that made most of its last N accesses

    @property
    def tiles(self) -> int:
        return self.width * self.height

    def tables(self):
        """(shared table, private table) as uint32 arrays of ZIPF_K + 1 entries."""
        zs = zipf_table(self.shared_lines, self.zipf_shared_s)
        zp = zipf_table(self.private_lines, self.zipf_private_s) if self.private_lines > 0 else zs
        return zs, zp

    def with_(self, **kw) -> "SimParams":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


def config0() -> SimParams:
    """4x4 mesh, background traffic at 0.05 flits/tile/cycle plus cache traffic over a
    shared Zipf(0.8) region of 2^20 lines, seed 1."""
    return SimParams(width=4, height=4, seed=1, bg_thr=thr(0.05), shared_lines=2**20,
                     private_lines=0, zipf_shared_s=0.8)


def config1() -> SimParams:
    """64x64 mesh, cache-driven traffic only: 30% shared Zipf(0.9) over 2^24 lines,
    70% private Zipf(0.9) over 2^14 lines per tile, seed 7."""
    return SimParams(width=64, height=64, seed=7, bg_thr=0, shared_thr=thr(0.3),
                     shared_lines=2**24, private_lines=2**14, zipf_shared_s=0.9,
                     zipf_private_s=0.9)


CONFIG2_RATES = (0.01, 0.05, 0.1, 0.2, 0.3)


def config2(rate: float = 0.05) -> SimParams:
    """208x208 mesh (43,264 tiles): the config-1 cache model plus uniform background
    traffic at `rate` flits/tile/cycle."""
    return config1().with_(width=208, height=208, bg_thr=thr(rate))


BATCH_SIDES = (8, 16, 24, 32, 48, 64)


def config3(n: int = 256, host_seed: int = 3) -> list[SimParams]:
    """Batch of n independent instances: sides drawn from BATCH_SIDES, background rate
    threshold integer-uniform in [thr(0.01), thr(0.3)], instance seed 1000 + i."""
    rng = np.random.Generator(np.random.PCG64(host_seed))
    sides = rng.choice(np.array(BATCH_SIDES), size=n)
    rates = rng.integers(thr(0.01), thr(0.3), endpoint=True, size=n)
    base = config1()
    return [base.with_(width=int(s), height=int(s), seed=1000 + i, bg_thr=int(r))
            for i, (s, r) in enumerate(zip(sides, rates))]


@dataclass(frozen=True)
class Job:
    """One served simulation job."""
    index: int
    arrival_s: float
    cycles: int
    params: SimParams


def config4(n_jobs: int, rate_per_s: float = 50.0, seed: int = 4,
            side_range=(4, 128), cycle_range=(10_000, 200_000)) -> list[Job]:
    """Poisson arrivals of jobs with side uniform in side_range and cycle counts
    log-uniform in cycle_range; each job runs the config-1 model with seed 100000 + j."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    t = np.cumsum(gaps)
    sides = rng.integers(side_range[0], side_range[1], endpoint=True, size=n_jobs)
    lo, hi = math.log(cycle_range[0]), math.log(cycle_range[1])
    cyc = np.exp(rng.uniform(lo, hi, size=n_jobs)).astype(np.int64)
    base = config1()
    return [Job(j, float(t[j]), int(cyc[j]),
                base.with_(width=int(sides[j]), height=int(sides[j]), seed=100000 + j))
            for j in range(n_jobs)]
