"""Serving loop: simulation jobs admitted as they arrive, run with continuous batching.

Each job is one chip (its own device buffer).  A job is admitted when its buffer fits the
HBM state budget and a slot is free, and its chip joins one resident batch (`simb_add`);
every scheduler tick advances all resident jobs together (`simb_step`: the patches of all
resident chips in one persistent launch, or a few launch groups when they do not fit the
device at once, each chip with its own remaining cycle count), retires the jobs that
finished (`simb_remove`), reads their statistics, frees their memory and admits new
arrivals.  A job whose creation or step fails is retired with its error; the
others keep running.  Requests that arrive while others run join at the
next tick, so their work overlaps on the device.  Because every chip's randomness is keyed
by its own (seed; cycle, tile), a job's result does not depend on what it ran beside.

The scheduler is written against a small backend interface so that its admission, memory
accounting and completion logic can be tested on the CPU with a stand-in backend.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np


@dataclass
class JobResult:
    index: int
    arrival_s: float
    admit_s: float
    finish_s: float
    cycles: int
    tiles: int
    stats: Optional[np.ndarray]
    error: Optional[str] = None

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s


class Backend:
    """What the scheduler needs from a simulator."""

    def state_bytes(self, params) -> int: ...
    def create(self, params): ...
    def step(self, chips: list, cycles: list[int]) -> None: ...
    def step_one(self, chip, cycles: int) -> None: ...
    def cycle(self, chip) -> int: ...
    def check(self, chip) -> None: ...
    def stats(self, chip) -> np.ndarray: ...
    def release(self, chip) -> None: ...


class GpuBackend(Backend):
    """Chips on the GPU through the C ABI, all members of one resident batch: a job's chip joins
    the batch when it is admitted (simb_add) and leaves when it retires (simb_remove); each
    tick is one simb_step over the members.  The launch table is sized once for `max_chips`
    chips of up to `max_patches` patches in all."""

    def __init__(self, block: int = 256, chunk: int = 1000, max_chips: int = 512, max_patches: int = 65536,
                 graph: bool = False):
        from paper_1508_03235_amd import nocsim
        self.nocsim = nocsim
        self.block = block
        self.chunk = chunk
        self.max_chips = max_chips
        self.max_patches = max_patches
        self.graph = graph
        self.batch = None

    def _batch(self):
        if self.batch is None:
            self.batch = self.nocsim.Batch((), block=self.block, max_chips=self.max_chips,
                                           max_patches=self.max_patches, graph=self.graph)
        return self.batch

    def state_bytes(self, params) -> int:
        return self.nocsim.state_bytes(params) + 256

    def create(self, params):
        s = self.nocsim.Sim(params)
        side = 16 if params.tiles > self.block else max(params.width, params.height)
        try:
            s.set_launch(min(side, params.width), min(side, params.height), self.block, self.chunk)
            self._batch().add(s)
        except Exception:
            s.close()
            raise
        return s

    def step(self, chips, cycles):
        b = self._batch()
        b.step({b.slot_of[id(c)]: int(n) for c, n in zip(chips, cycles)})

    def step_one(self, chip, cycles):
        chip.step(int(cycles))

    def cycle(self, chip):
        return chip.cycle

    def check(self, chip):
        chip.sync()

    def stats(self, chip):
        return chip.stats()

    def release(self, chip):
        if self.batch is not None and id(chip) in self.batch.slot_of:
            self.batch.remove(chip)
        chip.close()
        del chip.mem

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None


@dataclass
class _Live:
    job: object
    chip: object
    remaining: int
    admit_s: float
    nbytes: int


@dataclass
class ServeReport:
    results: list
    wall_s: float
    tile_cycles: int
    peak_bytes: int
    ticks: int

    def latency_percentiles(self):
        lat = np.array([r.latency_s for r in self.results if r.error is None])
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    @property
    def tile_cycles_per_s(self) -> float:
        return self.tile_cycles / self.wall_s if self.wall_s > 0 else 0.0


class Server:
    """Continuous-batching scheduler over a Backend.

    budget_bytes: device-state budget across resident jobs.  max_slots: resident jobs at once.
    tick_cycles: cycles each resident job advances per tick (or fewer if it finishes).
    clock: time source; `realtime=False` replays arrivals on a virtual clock that advances by
    the measured duration of each tick (so a run does not sleep through idle gaps).
    """

    def __init__(self, backend: Backend, budget_bytes: int, max_slots: int = 512,
                 tick_cycles: int = 2000, realtime: bool = False,
                 clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.tick_cycles = tick_cycles
        self.realtime = realtime
        self.clock = clock

    def run(self, jobs, on_finish=None) -> ServeReport:
        pending = sorted(jobs, key=lambda j: j.arrival_s)
        for j in pending:
            if self.backend.state_bytes(j.params) > self.budget:
                raise ValueError(f"job {j.index} needs more than the whole budget")
        arrivals = list(pending)
        arrivals.reverse()           # pop() gives the earliest
        waiting: list = []           # arrived, not admitted (FIFO)
        live: list[_Live] = []
        used = 0
        peak = 0
        results = []
        tile_cycles = 0
        ticks = 0
        t_start = self.clock()
        vnow = 0.0                   # virtual time since start

        def now():
            return self.clock() - t_start if self.realtime else vnow

        while arrivals or waiting or live:
            t = now()
            while arrivals and arrivals[-1].arrival_s <= t:
                waiting.append(arrivals.pop())
            if not live and not waiting and arrivals:
                # idle: jump (or sleep) to the next arrival
                nxt = arrivals[-1].arrival_s
                if self.realtime:
                    time.sleep(max(0.0, nxt - t))
                else:
                    vnow = nxt
                continue
            # admit in arrival order while memory and slots allow (no overtaking)
            while waiting and len(live) < self.max_slots:
                j = waiting[0]
                nb = self.backend.state_bytes(j.params)
                if used + nb > self.budget:
                    break
                waiting.pop(0)
                try:
                    chip = self.backend.create(j.params)
                except Exception as e:  # the job fails alone
                    results.append(JobResult(j.index, j.arrival_s, now(), now(), 0, j.params.tiles, None, repr(e)))
                    continue
                used += nb
                peak = max(peak, used)
                live.append(_Live(j, chip, j.cycles, now(), nb))
            if not live:
                continue
            # one tick: every resident job advances together
            steps = [min(self.tick_cycles, lv.remaining) for lv in live]
            t0 = self.clock()
            failed = {}
            before = [self.backend.cycle(lv.chip) for lv in live]
            try:
                self.backend.step([lv.chip for lv in live], steps)
            except Exception:
                # find the failing chips: finish each chip's share alone if the batch did not run
                # it, then check the chip's own error status
                for k, lv in enumerate(live):
                    try:
                        done = self.backend.cycle(lv.chip) - before[k]
                        if done < steps[k]:
                            self.backend.step_one(lv.chip, steps[k] - done)
                        self.backend.check(lv.chip)
                    except Exception as e:
                        failed[k] = repr(e)
            dt = self.clock() - t0
            if not self.realtime:
                vnow += dt
            ticks += 1
            for k, (lv, n) in enumerate(zip(live, steps)):
                if k in failed:
                    continue
                lv.remaining -= n
                tile_cycles += n * lv.job.params.tiles
            still = []
            for k, lv in enumerate(live):
                if k in failed:
                    results.append(JobResult(lv.job.index, lv.job.arrival_s, lv.admit_s, now(), lv.job.cycles - lv.remaining,
                                             lv.job.params.tiles, None, failed[k]))
                    self.backend.release(lv.chip)
                    used -= lv.nbytes
                elif lv.remaining == 0:
                    st = self.backend.stats(lv.chip)
                    r = JobResult(lv.job.index, lv.job.arrival_s, lv.admit_s, now(), lv.job.cycles,
                                  lv.job.params.tiles, st)
                    if on_finish:
                        on_finish(r, lv.chip)
                    results.append(r)
                    self.backend.release(lv.chip)
                    used -= lv.nbytes
                else:
                    still.append(lv)
            live = still
        wall = now()
        results.sort(key=lambda r: r.index)
        return ServeReport(results, wall, tile_cycles, peak, ticks)
