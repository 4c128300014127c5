"""Full-length runs of every workload configuration against results the serial oracle alone
computed (tests/golden/full_runs.json, written by tests/golden/make_goldens.py).

CPU tests check that the stored runs still describe today's workload generators (a change
there would make the stored hashes meaningless).  GPU tests run each configuration for its full
length in the build the benchmark times (no per-cycle digests) and compare the final canonical
state, then again in the checking build and compare the per-cycle state digests block by block.
"""
import json
import os

import numpy as np
import pytest

from paper_1508_03235_amd import workload as W

GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_runs.json")


def gold():
    with open(GOLD_PATH) as f:
        return json.load(f)


def h128(a):
    import xxhash
    return xxhash.xxh3_128_hexdigest(memoryview(np.ascontiguousarray(a)))


def params_of(run):
    return W.SimParams(**run["params"])


def variant_params():
    """The 208x208 variant runs (the benchmark's variants leg at background 0.05)."""
    base = W.config2(0.05)
    return {
        "config2_0.05_lspd": base.with_(flags=W.LSPD),
        "config2_0.05_lspd_central": base.with_(flags=W.LSPD | W.LSPD_CENTRAL),
        "config2_0.05_lspd_mig1": base.with_(flags=W.LSPD, mig_threshold=1),
        "config2_0.05_variants": base.with_(flags=W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY),
        "config2_0.05_rdelay2": base.with_(router_delay=2),
    }


# ---- CPU: the stored runs are the workloads of today -------------------------------------------

def test_golden_runs_match_workloads():
    g = gold()["runs"]
    assert params_of(g["config1"]) == W.config1() and g["config1"]["cycles"] == 100_000
    for r in W.CONFIG2_RATES:
        run = g[f"config2_{r}"]
        assert params_of(run) == W.config2(r) and run["cycles"] == 50_000
        assert len(run["digest_blocks"]) == 50
    assert len(g["config2_0.05"]["dumps"]) == 50      # every 1,000 cycles: the benchmark's timed runs
    c3 = W.config3()
    for i, p in enumerate(c3):
        run = g[f"config3_{i}"]
        assert params_of(run) == p and run["cycles"] == 20_000
    jobs = {j.index: j for j in W.config4(gold()["config4_sample"]["jobs_listed"])}
    keys = [k for k in g if k.startswith("config4_")]
    assert len(keys) == gold()["config4_sample"]["sample"]
    for k in keys:
        j = jobs[int(k.split("_")[1])]
        assert params_of(g[k]) == j.params and g[k]["cycles"] == j.cycles
    for k, p in variant_params().items():
        assert params_of(g[k]) == p and g[k]["cycles"] == 10_000 and len(g[k]["digest_blocks"]) == 10


def test_golden_hashes_are_xxh3_of_dump_bytes():
    """The hash convention the GPU tests use, on a dump the oracle writes here (4x4, 300 cycles
    against a fresh oracle run of the same cycles)."""
    from oracle import oracle as O
    p = W.config0()
    a, b = O.OracleSim(p), O.OracleSim(p)
    a.step(300)
    b.step(100)
    b.step(200)
    assert h128(a.dump().astype("<i4")) == h128(b.dump().astype("<i4"))


# ---- GPU: full-length parity in the timed build and in the checking build -----------------------

def gpu_run(p, cycles, chunk=10_000):
    """No-digest run (the timed build) of `cycles` cycles in chunks; returns the Sim."""
    from paper_1508_03235_amd import nocsim
    s = nocsim.Sim(p)
    done = 0
    while done < cycles:
        n = min(chunk, cycles - done)
        s.step(n)
        done += n
    return s


def digest_blocks(p, cycles, block):
    from paper_1508_03235_amd import nocsim
    s = nocsim.Sim(p)
    out, done = [], 0
    while done < cycles:
        n = min(block, cycles - done)
        out.append(h128(s.step(n, digests=True).astype("<u8")))
        done += n
    return out


@pytest.mark.gpu
def test_config1_full_length():
    run = gold()["runs"]["config1"]
    p = params_of(run)
    s = gpu_run(p, run["cycles"])
    assert h128(s.dump().astype("<i4")) == run["dumps"][str(run["cycles"])]
    del s
    assert digest_blocks(p, run["cycles"], 1000) == run["digest_blocks"]


@pytest.mark.gpu
@pytest.mark.parametrize("rate", W.CONFIG2_RATES)
def test_config2_full_length(rate):
    run = gold()["runs"][f"config2_{rate}"]
    p = params_of(run)
    s = gpu_run(p, run["cycles"])
    assert h128(s.dump().astype("<i4")) == run["dumps"][str(run["cycles"])]
    del s
    blocks = digest_blocks(p, run["cycles"], 1000)
    bad = [i for i, (a, b) in enumerate(zip(blocks, run["digest_blocks"])) if a != b]
    assert not bad, f"first differing block of 1,000 cycles: {bad[0]}"


@pytest.mark.gpu
@pytest.mark.parametrize("key", list(variant_params()))
def test_config2_variants_full_length(key):
    """The 208x208 chip under each variant (directory, central directory, migration, the router
    variants, router delay 2) for 10,000 cycles, on the kernel each runs on by default: final
    state in the timed build, per-cycle digests in the checking build."""
    run = gold()["runs"][key]
    p = params_of(run)
    s = gpu_run(p, run["cycles"])
    assert h128(s.dump().astype("<i4")) == run["dumps"][str(run["cycles"])]
    del s
    blocks = digest_blocks(p, run["cycles"], 1000)
    bad = [i for i, (a, b) in enumerate(zip(blocks, run["digest_blocks"])) if a != b]
    assert not bad, f"first differing block of 1,000 cycles: {bad[0]}"


@pytest.mark.gpu
def test_config2_intermediate_dumps_in_thousand_cycle_steps():
    """The benchmark's timed chip after whole 1,000-cycle steps (its launch chunk), compared at
    several step counts, including the default warmup + steps."""
    run = gold()["runs"]["config2_0.05"]
    p = params_of(run)
    from paper_1508_03235_amd import nocsim
    s = nocsim.Sim(p)
    for k in range(1, 21):
        s.step(1000)
        if k in (1, 3, 12, 20):
            assert h128(s.dump().astype("<i4")) == run["dumps"][str(1000 * k)], f"after {k} steps"


@pytest.mark.gpu
@pytest.mark.parametrize("graph", [False, True])
def test_config3_batch_full_length(graph):
    """All 256 instances in one batch (16x16-tile patches, 256-thread workgroups, as the
    benchmark times it), 20,000 cycles: every instance's final state equals its oracle run."""
    from paper_1508_03235_amd import nocsim
    g = gold()["runs"]
    params = W.config3()
    sims = [nocsim.Sim(p) for p in params]
    for s, p in zip(sims, params):
        side = min(16, p.width)
        s.set_launch(side, side, 256, 0)
    b = nocsim.Batch(sims, block=256, graph=graph)
    b.step(10_000)
    b.step(10_000)
    b.close()
    bad = [i for i, s in enumerate(sims) if h128(s.dump().astype("<i4")) != g[f"config3_{i}"]["dumps"]["20000"]]
    assert not bad, f"instances differing from the oracle: {bad[:10]}"


@pytest.mark.gpu
def test_config4_sampled_jobs_full_length():
    """The sampled served jobs, each run for its full cycle count in one batch (as the serving
    loop runs them: 256-thread workgroups, 1,000-cycle chunks), against their oracle runs."""
    from paper_1508_03235_amd import nocsim
    g = gold()["runs"]
    keys = sorted(k for k in g if k.startswith("config4_"))
    sims = [nocsim.Sim(params_of(g[k])) for k in keys]
    for s in sims:   # the serving backend's mapping: 16x16-tile patches, or the whole chip if it fits
        pp = s.params
        side = 16 if pp.tiles > 256 else max(pp.width, pp.height)
        s.set_launch(min(side, pp.width), min(side, pp.height), 256, 1000)
    b = nocsim.Batch(sims, block=256)
    b.step([g[k]["cycles"] for k in keys])
    b.close()
    for k, s in zip(keys, sims):
        assert s.cycle == g[k]["cycles"]
        assert h128(s.dump().astype("<i4")) == g[k]["dumps"][str(g[k]["cycles"])], k


@pytest.mark.gpu
def test_config3_batch_full_length_on_tuned_mapping():
    """The batch autotuner's patch shapes (as the benchmark times the batch): all 256 instances,
    20,000 cycles, equal to their oracle runs."""
    from paper_1508_03235_amd import autotune, nocsim
    g = gold()["runs"]
    params = W.config3()
    mapping, rate, trials = autotune.tune_batch(params, block=256, cycles=300, warmup=50)
    assert trials > 1 and rate > 0
    assert all(pw * ph <= 256 for pw, ph in mapping.values())
    sims = [nocsim.Sim(p) for p in params]
    autotune.apply_batch_mapping(sims, mapping, block=256)
    b = nocsim.Batch(sims, block=256)
    b.step(20_000)
    b.close()
    bad = [i for i, s in enumerate(sims) if h128(s.dump().astype("<i4")) != g[f"config3_{i}"]["dumps"]["20000"]]
    assert not bad, f"instances differing from the oracle: {bad[:10]}"
