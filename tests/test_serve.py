"""Serving loop: admission by memory budget, continuous batching, and per-job results that
do not depend on the mix (oracle backend on the CPU; GPU backend under -m gpu)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from paper_1508_03235_amd.serve import GpuBackend, Server
from fake_backend import OracleBackend


def small_jobs(n, seed=4):
    jobs = W.config4(n, rate_per_s=2000.0, seed=seed, side_range=(2, 6), cycle_range=(50, 400))
    # keep the oracle cheap: small caches
    return [W.Job(j.index, j.arrival_s, j.cycles,
                  j.params.with_(l1_sets=8, l1_ways=2, l2_sets=16, l2_ways=4, mem_lat=20))
            for j in jobs]


def alone(job):
    o = O.OracleSim(job.params)
    o.step(job.cycles)
    return o.dump(), o.stats()


def test_oracle_backend_every_job_equals_its_solo_run():
    jobs = small_jobs(24)
    be = OracleBackend()
    budget = 5 * max(be.state_bytes(j.params) for j in jobs)
    dumps = {}
    rep = Server(be, budget, tick_cycles=64).run(jobs, on_finish=lambda r, chip: dumps.__setitem__(r.index, chip.dump()))
    assert len(rep.results) == len(jobs)
    assert rep.peak_bytes <= budget
    assert rep.tile_cycles == sum(j.cycles * j.params.tiles for j in jobs)
    for j, r in zip(jobs, rep.results):
        d, st = alone(j)
        assert r.index == j.index and r.cycles == j.cycles
        assert (r.stats == st).all(), j.index
        assert (dumps[j.index] == d).all(), j.index
        assert r.admit_s >= r.arrival_s and r.finish_s >= r.admit_s


def test_budget_forces_queueing_in_arrival_order():
    # jobs of one size, and a budget of exactly one job: never two resident at once
    jobs = [W.Job(j.index, j.arrival_s, j.cycles, j.params.with_(width=4, height=4)) for j in small_jobs(10)]
    be = OracleBackend()
    budget = be.state_bytes(jobs[0].params)
    rep = Server(be, budget, tick_cycles=1000).run(jobs)
    order = sorted(rep.results, key=lambda r: r.admit_s)
    assert [r.index for r in order] == sorted(r.index for r in rep.results)
    for a, b in zip(order, order[1:]):
        assert b.admit_s >= a.finish_s   # no overlap when only one fits
    p50, p99 = rep.latency_percentiles()
    assert p99 >= p50 > 0


def test_job_larger_than_budget_is_rejected():
    jobs = small_jobs(2)
    with pytest.raises(ValueError):
        Server(OracleBackend(), budget_bytes=10).run(jobs)


class FlakyBackend(OracleBackend):
    """The oracle backend with one job that cannot be created and one chip whose step fails."""

    def __init__(self, bad_create, bad_step):
        super().__init__()
        self.bad_create, self.bad_step = bad_create, bad_step

    def create(self, params):
        if params.seed == self.bad_create:
            raise RuntimeError("no memory for this job")
        return super().create(params)

    def step(self, chips, cycles):
        if any(c.params.seed == self.bad_step for c in chips):
            raise RuntimeError("batch step failed")
        super().step(chips, cycles)

    def step_one(self, chip, cycles):
        if chip.params.seed == self.bad_step:
            raise RuntimeError("chip fault")
        super().step_one(chip, cycles)


def test_failures_are_isolated_per_job():
    jobs = small_jobs(12)
    be = FlakyBackend(bad_create=jobs[3].params.seed, bad_step=jobs[7].params.seed)
    budget = 4 * max(be.state_bytes(j.params) for j in jobs)
    dumps = {}
    rep = Server(be, budget, tick_cycles=50).run(jobs, on_finish=lambda r, chip: dumps.__setitem__(r.index, chip.dump()))
    by = {r.index: r for r in rep.results}
    assert len(by) == len(jobs)
    assert by[3].error and "no memory" in by[3].error
    assert by[7].error and "chip fault" in by[7].error
    for j in jobs:
        if j.index in (3, 7):
            continue
        assert by[j.index].error is None
        d, st = alone(j)
        assert (dumps[j.index] == d).all(), j.index   # neighbours of the failing chip are unaffected


@pytest.mark.gpu
def test_gpu_serving_results_equal_solo_runs():
    from paper_1508_03235_amd import nocsim
    jobs = W.config4(12, rate_per_s=500.0, seed=9, side_range=(4, 24), cycle_range=(200, 1500))
    be = GpuBackend(block=256, chunk=500)
    dumps = {}
    rep = Server(be, budget_bytes=8 << 30, tick_cycles=300).run(
        jobs, on_finish=lambda r, chip: dumps.__setitem__(r.index, chip.dump()))
    assert len(rep.results) == len(jobs)
    assert rep.ticks > 1
    for j in jobs:
        d, _ = alone(j)
        assert (dumps[j.index] == d).all(), f"job {j.index} differs from the oracle"
        g = nocsim.Sim(j.params)
        g.step(j.cycles)
        assert (g.dump() == d).all()
