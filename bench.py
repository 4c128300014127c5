"""Benchmark: simulated tile-cycles per second of the 208x208 (43,264-tile) chip.

One step = 1,000 simulated cycles of the whole per-cycle path (memory access at L1 and the
home L2 slice, oldest-first deflection arbitration, traversal/ejection/injection) over every
tile, running the config-1 cache model plus uniform background traffic at 0.05 flits per
tile per cycle (a saturated point of the paper-style sweep).  Inputs are synthetic and seeded
(workload module); all state is resident in HBM before the timed region starts.

Besides the headline line the JSON carries:
  roofline     - algorithmic bytes per launch of the step kernel / its measured duration,
                 against the 8 TB/s HBM peak;
  cpu_baseline - the serial oracle on the host, on a bounded prefix of the same workload;
  parity       - per-cycle state digests of a GPU run compared with the oracle on that
                 prefix, and the timed chip's own final state compared with the oracle's state
                 after the same cycles (stored oracle runs); `checked` is true only when the
                 latter matched;
  oracle_configs - the serial oracle timed on every workload configuration (one pinned host
                 thread each) and on all host CPUs at once for configs 2 and 3;
  sweep        - per-rate throughput and the sweep's outputs (deflection rate, average
                 latency, L2 hit rate) (skip with --no-sweep);
  packets      - the same chip with replies of 4 flits (the paper's Table 1, remote L2 access):
                 throughput, flit and op latency against single-flit replies, and per-cycle
                 digests of a prefix against the oracle (--no-packets);
  variants     - the same chip under each model variant (priority by deflection count, hit
                 under miss, injection register, all three; router delay 2; the LSPD directory,
                 interleaved and central, and migrating a block on every remote access) on the general
                 kernel, beside the base model on that kernel, and each again on the
                 one-tile-per-thread kernel: throughput, deflection rate, latencies, ops per
                 tile-cycle, and per-cycle digests of a prefix against the oracle (--no-variants);
  meshes       - square meshes from 208x208 to 832x832 tiles on their default mapping:
                 throughput, kernel and device state (--no-meshes);
  batched      - the 256-chip batch in one launch per chunk, on the batch autotuner's patch shapes,
                 vs the same chips run one at a time on the single-chip autotuner's mappings
                 (--no-batched);
  serving      - Poisson-arriving simulation jobs under continuous batching: p50/p99 job
                 latency and aggregate throughput, against one job at a time (--no-serving).
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

HBM_PEAK_GBS = 8000.0
CYCLES_PER_STEP = 1000


def algorithmic_bytes(p, st_delta, cycles):
    """Bytes a cycle sweep must move at least, counted from the run's own events:
    per directed link, its 4-byte destination word read as an input and written as an output
    (8 B), plus the 12 payload bytes of each occupied slot written by the sender and read by
    the receiver (24 B per traversal); the core's 8-byte state read and written (16 B per
    tile-cycle); 20 B read and 8 B written per issued op at L1 (the 4-way set and its order);
    36 B read and 8 B written per L2 lookup (the 8-way set); 12 B per reply-queue node
    operation (append at a request's arrival, pop at a reply's departure)."""
    W, H = p.width, p.height
    N = W * H
    links = 4 * N - 2 * W - 2 * H
    from paper_1508_03235_amd.nocsim import STAT
    g = lambda k: int(st_delta[STAT[k]])
    b = cycles * (links * 8 + N * 16)
    b += g("traversals") * 24
    b += g("ops_issued") * 28
    b += (g("l2_hit") + g("l2_miss")) * 44
    b += (g("req_received") + g("reply_sent")) * 12
    return b


def event_bytes(p, st_delta, cycles):
    """A wider count kept beside the headline one: the whole 13-word core record read every
    tile-cycle, 16 B per injection, ejection and op event, L1 and L2 sets read and written in
    full on every access, 12 B per queue append and 8 B per pop."""
    W, H = p.width, p.height
    N = W * H
    links = 4 * N - 2 * W - 2 * H
    from paper_1508_03235_amd.nocsim import STAT
    g = lambda k: int(st_delta[STAT[k]])
    inj = g("inj_req") + g("inj_reply") + g("inj_bg")
    ej = g("ej_req") + g("ej_reply") + g("ej_bg")
    b = cycles * (links * 8 + N * 52)
    b += g("traversals") * 24
    b += (inj + ej + g("ops_issued") + g("ops_done")) * 16
    b += (g("ops_issued") + g("ops_done")) * 2 * 16
    b += (g("l2_hit") + g("l2_miss")) * 2 * 32
    b += g("req_received") * 12 + g("reply_sent") * 8
    return b


def kernel_events_ms(e0, e1, n_cycles, chunk):
    """Average duration of one step-kernel launch over a region bracketed by events e0, e1 on
    the chip's stream (n_cycles cycles in launches of `chunk` cycles)."""
    launches = -(-n_cycles // chunk)
    return e0.elapsed_time(e1) / launches, launches


def profiled_traffic(kernel_tag):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a copy
    calibration) for this exact kernel build (source and compiler flags), or None when either
    changed since."""
    import re
    from __graft_entry__ import build_signature
    prof = os.path.join(ROOT, "profiles", f"{kernel_tag}_208x208_bg0.05_counters.md")
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    m_sha = re.search(r"kernel build sha256 \(source and compiler flags, first 16 hex\): ([0-9a-f]{16})", text)
    m_b = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_sha or not m_b or m_sha.group(1) != build_signature():
        return None
    return int(m_b.group(1))


def host_cpu():
    """Host CPU description: logical CPUs the process may use, and the model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


class pinned:
    """Pins the calling thread to one host CPU for the duration of a with-block."""

    def __init__(self, cpu=None):
        self.cpu = cpu

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        cpu = self.cpu if self.cpu is not None else min(self.saved)
        os.sched_setaffinity(0, {cpu})
        return cpu

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)


def cpu_baseline(p, budget_s=12.0):
    from oracle import oracle as O
    O.build()
    o = O.OracleSim(p)
    with pinned() as cpu:
        t0 = time.perf_counter()
        n = 0
        digests = []
        while time.perf_counter() - t0 < budget_s:
            digests.append(o.step(50, digests=True))
            n += 50
        dt = time.perf_counter() - t0
    o.close()
    host = host_cpu()
    return {"value": p.tiles * n / dt, "unit": "tile-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{p.width}x{p.height} chip, first {n} cycles of the benchmark workload, "
                      f"serial C oracle (gcc -O3), one host thread pinned to CPU {cpu}, {dt:.1f} s",
            "host": host}, np.concatenate(digests)


def _oracle_worker(task):
    """(params dict, seconds, cpu) -> (tile-cycles, seconds): the oracle on one pinned CPU."""
    pd, budget, cpu = task
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_1508_03235_amd.workload import SimParams
    if cpu is not None:
        os.sched_setaffinity(0, {cpu})
    p = SimParams(**pd)
    o = O.OracleSim(p)
    t0 = time.perf_counter()
    n = 0
    step = max(1, min(1000, int(2e6 // p.tiles)))
    while time.perf_counter() - t0 < budget:
        o.step(step)
        n += step
    dt = time.perf_counter() - t0
    o.close()
    return p.tiles * n, dt


def oracle_configs(W, budget=2.0, max_procs=16):
    """The serial oracle on every workload configuration: one pinned host thread per config
    (bounded samples of `budget` seconds), and for the multi-run configurations (config 2's five
    rates, config 3's instances) independent oracle processes on all host CPUs at once (at most
    `max_procs`), reported as their aggregate tile-cycles/s."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    cpus = sorted(os.sched_getaffinity(0))
    procs = min(len(cpus), max_procs)
    c3 = W.config3()
    jobs = W.config4(60)
    single = {"config0": W.config0(), "config1": W.config1(), "config2_0.05": W.config2(0.05),
              "config3_instance0": c3[0], "config4_job0": jobs[0].params}
    out = {"host": host_cpu(), "budget_s_per_sample": budget, "single_core": {}, "all_core": {}}
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        for name, p in single.items():
            tc, dt = pool.apply(_oracle_worker, ((p.as_dict(), budget, cpus[0]),))
            out["single_core"][name] = {"tiles": p.tiles, "tile_cycles_per_s": tc / dt}
        for name, plist in (("config2_five_rates", [W.config2(r) for r in W.CONFIG2_RATES]),
                            ("config3_instances", c3[:procs])):
            tasks = [(q.as_dict(), budget, cpus[i % len(cpus)]) for i, q in enumerate(plist[:procs])]
            res = pool.map(_oracle_worker, tasks)
            out["all_core"][name] = {"processes": len(tasks),
                                     "tile_cycles_per_s": sum(tc / dt for tc, dt in res)}
    return out


def timed_run_check(sim, p, rate):
    """The timed chip's own state at the end of the timed region against the oracle's state after
    the same number of cycles (stored by tests/golden/make_goldens.py, which runs the oracle only)."""
    path = os.path.join(ROOT, "tests", "golden", "full_runs.json")
    if not os.path.exists(path):
        return {"checked": False, "reason": "no stored oracle runs"}
    with open(path) as f:
        run = json.load(f)["runs"].get(f"config2_{rate}")
    if run is None or run["params"] != p.as_dict():
        return {"checked": False, "reason": "no stored oracle run of this workload"}
    key = str(sim.cycle)
    if key not in run["dumps"]:
        return {"checked": False, "reason": f"no stored oracle state after {key} cycles"}
    import xxhash
    h = xxhash.xxh3_128_hexdigest(memoryview(np.ascontiguousarray(sim.dump().astype("<i4"))))
    return {"checked": True, "cycles": sim.cycle, "state_equal_oracle": h == run["dumps"][key]}


def run_sweep(nocsim, W, torch, cycles):
    out = []
    for rate in W.CONFIG2_RATES:
        p = W.config2(rate)
        sim = nocsim.Sim(p)
        sim.step(200)
        st0 = sim.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(cycles)
        dt = time.perf_counter() - t0
        st = sim.stats() - st0
        S = nocsim.STAT
        ej = st[S["ej_req"]] + st[S["ej_reply"]] + st[S["ej_bg"]]
        lat = st[S["lat_req"]] + st[S["lat_reply"]] + st[S["lat_bg"]]
        out.append({"rate": rate, "tile_cycles_per_s": p.tiles * cycles / dt,
                    "deflection_rate": float(st[S["deflections"]] / max(1, st[S["traversals"]])),
                    "avg_latency": float(lat / max(1, ej)),
                    "l2_hit_rate": float(st[S["l2_hit"]] / max(1, st[S["l2_hit"]] + st[S["l2_miss"]]))})
        del sim
    return out


def run_packets(nocsim, W, torch, O, cycles, parity_cycles=200, flits=4):
    """The 208x208 chip at background 0.05 with multi-flit replies, beside single-flit ones."""
    out = {"reply_flits": flits}
    for f in (1, flits):
        p = W.config2(0.05).with_(reply_flits=f)
        sim = nocsim.Sim(p)
        sim.step(500)
        st0 = sim.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(cycles)
        dt = time.perf_counter() - t0
        st = sim.stats() - st0
        S = nocsim.STAT
        ej = st[S["ej_req"]] + st[S["ej_reply"]] + st[S["ej_bg"]]
        lat = st[S["lat_req"]] + st[S["lat_reply"]] + st[S["lat_bg"]]
        out[f"flits_{f}"] = {"tile_cycles_per_s": p.tiles * cycles / dt,
                             "avg_flit_latency": float(lat / max(1, ej)),
                             "avg_op_latency": float(st[S["op_lat"]] / max(1, st[S["ops_done"]])),
                             "ops_per_tile_cycle": float(st[S["ops_done"]] / (p.tiles * cycles))}
        del sim
    if O is not None:
        p = W.config2(0.05).with_(reply_flits=flits)
        g = nocsim.Sim(p).step(parity_cycles, digests=True)
        o = O.OracleSim(p).step(parity_cycles, digests=True)
        out["parity"] = {"cycles": parity_cycles, "digests_equal": bool((g == o).all())}
    return out


def run_variants(nocsim, W, torch, O, cycles, parity_cycles=100, only=None):
    """The 208x208 chip at background 0.05 under each model variant, on the general kernel and
    on the one-tile-per-thread kernel."""
    out = {}
    cases = [("base", 0), ("age_deflect", W.AGE_DEFLECT), ("hit_under_miss", W.HIT_UNDER_MISS),
             ("inject_delay", W.INJECT_DELAY), ("all", W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY),
             ("router_delay_2", 0), ("lspd", W.LSPD), ("lspd_central", W.LSPD | W.LSPD_CENTRAL),
             ("lspd_migration_1", W.LSPD), ("age_deflect_fast", W.AGE_DEFLECT),
             ("hit_under_miss_fast", W.HIT_UNDER_MISS), ("inject_delay_fast", W.INJECT_DELAY),
             ("all_fast", W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY), ("router_delay_2_fast", 0),
             ("lspd_fast", W.LSPD), ("lspd_central_fast", W.LSPD | W.LSPD_CENTRAL), ("lspd_migration_1_fast", W.LSPD)]
    S = nocsim.STAT
    for name, flags in cases:
        if only and name not in only:
            continue
        generic = not name.endswith("_fast")
        p = W.config2(0.05).with_(flags=flags, router_delay=2 if name.startswith("router_delay_2") else 1,
                                  mig_threshold=1 if name.startswith("lspd_migration_1") else 0)
        sim = nocsim.Sim(p)
        sim.set_kernel(generic)
        sim.step(300)
        st0 = sim.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(cycles)
        dt = time.perf_counter() - t0
        st = sim.stats() - st0
        ej = st[S["ej_req"]] + st[S["ej_reply"]] + st[S["ej_bg"]]
        lat = st[S["lat_req"]] + st[S["lat_reply"]] + st[S["lat_bg"]]
        r = {"flags": flags, "router_delay": p.router_delay, "kernel": "general" if generic else "one tile per thread",
             "state_gb": nocsim.state_bytes(p) / 1e9,  # the chip's device state (the model's memory cost)
             "tile_cycles_per_s": p.tiles * cycles / dt,
             "deflection_rate": float(st[S["deflections"]] / max(1, st[S["traversals"]])),
             "avg_flit_latency": float(lat / max(1, ej)),
             "max_flit_latency": int(sim.stats()[S["lat_max"]]),
             "avg_op_latency": float(st[S["op_lat"]] / max(1, st[S["ops_done"]])),
             "ops_per_tile_cycle": float(st[S["ops_done"]] / (p.tiles * cycles))}
        if flags & W.LSPD:
            r["directory"] = {k: int(st[S[k]]) for k in ("dir_access", "dir_nack", "trap", "dir_evict", "l2_hit", "l2_miss",
                                                         "migrations", "redirects")}
        del sim
        if O is not None:
            g = nocsim.Sim(p)
            g.set_kernel(generic)
            r["parity"] = {"cycles": parity_cycles, "digests_equal": bool(
                (g.step(parity_cycles, digests=True) == O.OracleSim(p).step(parity_cycles, digests=True)).all())}
            del g
        out[name] = r
    return out


def run_meshes(nocsim, W, torch, cycles, sides=(208, 256, 320, 416, 624, 832)):
    """Square meshes of growing size (the config-2 model at background 0.05, 2^10 private lines
    per tile so that every line stays below 2^30) on the default mapping: throughput, the
    kernel it runs on and the device state."""
    out = {}
    for side in sides:
        p = W.config2(0.05).with_(width=side, height=side, private_lines=2**10)
        sim = nocsim.Sim(p)
        pw, ph, block, chunk = sim.get_launch()
        sim.step(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(cycles)
        dt = time.perf_counter() - t0
        out[f"{side}x{side}"] = {"tiles": p.tiles, "patch": [pw, ph], "block": block,
                                 "kernel": "one tile per thread" if pw * ph <= block else "general",
                                 "tile_cycles_per_s": p.tiles * cycles / dt, "us_per_cycle": dt / cycles * 1e6,
                                 "state_gb": nocsim.state_bytes(p) / 1e9}
        del sim
    return out


def run_batched(nocsim, W, torch, cycles, plain_chips=None):
    """Config 3: the 256 uneven chips in one batch, each chip shape on the patch shape the batch
    autotuner picked, against the same chips run one at a time, each on the best single-chip
    mapping the single-chip autotuner found for its shape (all 256, or the first `plain_chips`)."""
    from paper_1508_03235_amd import autotune
    params = W.config3()
    mapping, tuned_rate, trials = autotune.tune_batch(params, block=256, cycles=1000, warmup=200)
    sims = [nocsim.Sim(p) for p in params]
    autotune.apply_batch_mapping(sims, mapping, block=256)
    b = nocsim.Batch(sims, block=256)
    b.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(cycles)
    dt = time.perf_counter() - t0
    tiles = sum(p.tiles for p in params)
    batched = tiles * cycles / dt
    b.close()
    del b, sims
    # one at a time, each chip on its shape's best single-chip mapping
    best = {}
    for p in params:
        key = (p.width, p.height)
        if key not in best:
            best[key] = autotune.tune(p, cycles=300, warmup=50, cache_path=None)
    sample = params if not plain_chips else params[:plain_chips]
    t_plain, tiles_plain = 0.0, 0
    for p in sample:
        s = nocsim.Sim(p)
        pw, ph, blk = best[(p.width, p.height)]
        s.set_launch(pw, ph, blk, 0)
        s.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(cycles)
        t_plain += time.perf_counter() - t0
        tiles_plain += p.tiles
        del s
    plain = tiles_plain * cycles / t_plain
    fmt = lambda m: {f"{w}x{h}": list(v) for (w, h), v in sorted(m.items())}
    return {"chips": len(params), "tiles": tiles, "cycles": cycles,
            "batched_tile_cycles_per_s": batched, "plain_tile_cycles_per_s": plain,
            "plain_chips": len(sample), "speedup": batched / plain,
            "batch_mapping_patch": fmt(mapping), "batch_tuner_trials": trials,
            "plain_mapping_patch_block": fmt(best)}


def run_serving(W, n_jobs, one_at_a_time_jobs):
    """Config 4: Poisson arrivals (50 jobs/s) of jobs with side U[4,128] and cycles
    log-U[1e4, 2e5], admitted under a 200 GB state budget, continuous batching; against the
    same arrival stream served one job at a time."""
    from paper_1508_03235_amd.serve import GpuBackend, Server
    jobs = W.config4(n_jobs)
    be = GpuBackend(block=256, chunk=1000)
    rep = Server(be, budget_bytes=200 << 30, tick_cycles=2000, realtime=True).run(jobs)
    p50, p99 = rep.latency_percentiles()
    out = {"jobs": n_jobs, "arrival_rate_per_s": 50.0, "budget_gb": 200,
           "tile_cycles_per_s": rep.tile_cycles_per_s, "p50_latency_s": p50, "p99_latency_s": p99,
           "wall_s": rep.wall_s, "ticks": rep.ticks, "peak_state_gb": rep.peak_bytes / 2**30}
    if one_at_a_time_jobs:
        sub = jobs[:one_at_a_time_jobs]
        rep1 = Server(be, budget_bytes=200 << 30, max_slots=1, tick_cycles=2000, realtime=True).run(sub)
        q50, q99 = rep1.latency_percentiles()
        rep2 = Server(be, budget_bytes=200 << 30, tick_cycles=2000, realtime=True).run(sub)
        r50, r99 = rep2.latency_percentiles()
        out["same_jobs"] = {"jobs": len(sub),
                            "one_at_a_time": {"tile_cycles_per_s": rep1.tile_cycles_per_s, "p50_latency_s": q50,
                                              "p99_latency_s": q99, "wall_s": rep1.wall_s},
                            "continuous_batching": {"tile_cycles_per_s": rep2.tile_cycles_per_s,
                                                    "p50_latency_s": r50, "p99_latency_s": r99, "wall_s": rep2.wall_s}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rate", type=float, default=0.05)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle-configs", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-packets", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant", action="append", default=None, metavar="NAME",
                    help="run only the named variant (repeatable), e.g. lspd_fast")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-meshes", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=60)
    ap.add_argument("--launch", type=str, default="", help="patch_w,patch_h,block,chunk")
    ap.add_argument("--maps-out", type=str, default="",
                    help="at interpreter exit, write this process's /proc/self/maps to the given file "
                         "(to symbolize addresses a crash report at process exit prints)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (scales the "
                         "profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.maps_out:
        import atexit

        def _dump_maps(path=args.maps_out):
            with open("/proc/self/maps") as src, open(path, "w") as dst:
                dst.write(src.read())
        atexit.register(_dump_maps)
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the simulator runs a chip on one GPU (sharding a chip "
              "across GPUs is a design, not built); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    from paper_1508_03235_amd import workload as W
    # oracle timings in worker processes first: started before this process touches the GPU
    oc = None
    if not args.no_cpu and not args.no_oracle_configs:
        try:
            oc = oracle_configs(W)
        except Exception as e:
            oc = {"error": repr(e)}
        print("# oracle timings done", file=sys.stderr, flush=True)

    import torch
    from paper_1508_03235_amd import nocsim

    torch.cuda.set_device(0)
    p = W.config2(args.rate)
    sim = nocsim.Sim(p)
    if args.launch:
        sim.set_launch(*[int(v) for v in args.launch.split(",")])
    pw, ph, block, chunk = sim.get_launch()
    print(f"# {p.width}x{p.height} chip, launch patch={pw}x{ph} block={block} chunk={chunk}", file=sys.stderr, flush=True)

    # parity on the benchmark configuration: digests of the first cycles vs the oracle
    cpu = None
    parity = None
    if not args.no_cpu:
        cpu, odig = cpu_baseline(p, args.cpu_budget)
        n_par = len(odig)
        chk = nocsim.Sim(p)
        chk.set_launch(pw, ph, block, chunk)
        gdig = chk.step(n_par, digests=True)
        parity = {"cycles": n_par, "digests_equal": bool((gdig == odig).all())}
        del chk
        print(f"# parity over {n_par} cycles: {parity['digests_equal']}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        sim.step(CYCLES_PER_STEP)
    torch.cuda.synchronize()
    st0 = sim.stats()
    # events on the chip's stream around the timed launches (the roofline's launch duration)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        sim.step(CYCLES_PER_STEP, sync=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.sync()
    st = sim.stats() - st0
    cycles = args.steps * CYCLES_PER_STEP
    value = p.tiles * cycles / dt
    # the timed run itself, checked against the oracle after the same cycles
    timed_check = timed_run_check(sim, p, args.rate)
    print(f"# timed run vs oracle: {timed_check}", file=sys.stderr, flush=True)

    # roofline of the step kernel: its launches in the timed region, event-timed on the chip's stream
    ms_launch, launches = kernel_events_ms(ev0, ev1, cycles, chunk)
    abytes_per_launch = algorithmic_bytes(p, st, cycles) / cycles * chunk
    achieved = abytes_per_launch / (ms_launch * 1e-3) / 1e9
    fast = pw * ph <= block
    kernel = "step_fast<true>" if fast else "step_kernel<true>"
    traffic = profiled_traffic("step_fast" if fast else "step_kernel") if (args.rate == 0.05 and not args.launch) else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kernel, "launch_ms": ms_launch, "cycles_per_launch": chunk,
            "algorithmic_bytes_per_tile_cycle": abytes_per_launch / chunk / p.tiles,
            "traffic_note": "HBM bytes per launch from rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0 "
                            "(profiles/, same hash of kernel source and compiler flags), null if either changed"}

    S = nocsim.STAT
    ej = st[S["ej_req"]] + st[S["ej_reply"]] + st[S["ej_bg"]]
    out = {
        "metric": "simulated tile-cycles/sec at ~43k-tile mesh, bit-exact vs oracle; batched vs plain",
        "value": value, "unit": "tile-cycles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"208x208 bufferless mesh (43,264 tiles), config-1 cache model + "
                               f"uniform background {args.rate} flits/tile/cycle, seed 7, "
                               f"{CYCLES_PER_STEP} cycles per step",
                   "tiles": p.tiles, "cycles_per_step": CYCLES_PER_STEP,
                   "launch": {"patch": [pw, ph], "block": block, "chunk": chunk}},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": {"prefix_digests": parity, "timed_run": timed_check},
        "checked": bool(timed_check.get("state_equal_oracle", False)),
        "run": {"deflection_rate": float(st[S["deflections"]] / max(1, st[S["traversals"]])),
                "avg_latency": float((st[S["lat_req"]] + st[S["lat_reply"]] + st[S["lat_bg"]]) / max(1, ej)),
                "l2_hit_rate": float(st[S["l2_hit"]] / max(1, st[S["l2_hit"]] + st[S["l2_miss"]]))},
    }
    if cpu:
        out["gpu_over_oracle"] = value / cpu["value"]
    if oc is not None:
        if "error" not in oc:
            oc["gpu_over_oracle_single_core"] = value / oc["single_core"]["config2_0.05"]["tile_cycles_per_s"]
            oc["gpu_over_oracle_all_core_config2"] = value / oc["all_core"]["config2_five_rates"]["tile_cycles_per_s"]
        out["oracle_configs"] = oc
    if not args.no_sweep:
        try:
            out["sweep"] = run_sweep(nocsim, W, torch, 5000)
        except Exception as e:  # an optional leg must not hide the headline number
            out["sweep"] = {"error": repr(e)}
    O = None  # the oracle checks the optional legs' prefixes when the CPU leg ran
    if cpu:
        from oracle import oracle as O
    if not args.no_packets:
        try:
            out["packets"] = run_packets(nocsim, W, torch, O, 5000)
        except Exception as e:
            out["packets"] = {"error": repr(e)}
    if not args.no_variants:
        try:
            out["variants"] = run_variants(nocsim, W, torch, O, 3000, only=args.variant)
        except Exception as e:
            out["variants"] = {"error": repr(e)}
    if not args.no_meshes:
        try:
            out["meshes"] = run_meshes(nocsim, W, torch, 500)
        except Exception as e:
            out["meshes"] = {"error": repr(e)}
    if not args.no_batched:
        try:
            out["batched"] = run_batched(nocsim, W, torch, 2000)
        except Exception as e:
            out["batched"] = {"error": repr(e)}
    if not args.no_serving:
        try:
            out["serving"] = run_serving(W, args.serving_jobs, one_at_a_time_jobs=12)
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
