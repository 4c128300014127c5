"""Parity of the model variants (SimParams.flags) on the GPU with the serial oracle.

Priority by deflection count, hit under miss, the injection register and the router delay
run on the one-tile-per-thread kernel as well as on the general one; the directory runs on
the general kernel.  Bar: bit-exact, as for the base model: every
per-cycle digest and the final canonical dump, including each in-flight flit's deflection
count and each core's held op.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import STAT, split_dump
from tests.test_gpu_parity import assert_same_run, gpu_sim

pytestmark = pytest.mark.gpu

AGE, HUM, DELAY = W.AGE_DEFLECT, W.HIT_UNDER_MISS, W.INJECT_DELAY
FLAG_SETS = [AGE, HUM, DELAY, AGE | HUM | DELAY]
IDS = ["age", "hum", "delay", "all"]


@pytest.mark.parametrize("flags", FLAG_SETS, ids=IDS)
def test_variants_config0_full_run(flags):
    """4x4, 10,000 cycles of config 0 under each variant."""
    assert_same_run(W.config0().with_(flags=flags, op_thr=W.thr(0.5)), 10_000, step_sizes=[1, 999, 4000, 5000])


@pytest.mark.parametrize("flags", FLAG_SETS, ids=IDS)
@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (5, 5), (13, 7)])
def test_variants_small_shapes(w, h, flags):
    p = W.config0().with_(width=w, height=h, seed=w * 100 + h + flags, bg_thr=W.thr(0.25) if w * h > 1 else 0,
                          op_thr=W.thr(0.6), l1_sets=8, l1_ways=2, shared_lines=256, flags=flags, reply_flits=2)
    assert_same_run(p, 3000)


@pytest.mark.parametrize("flags", [AGE, DELAY, AGE | DELAY, AGE | HUM | DELAY], ids=["age", "delay", "age_delay", "all"])
@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (7, 2, 64, 0), (20, 1, 64, 0), (5, 5, 64, 37), (20, 13, 64, 0)])
def test_variants_patch_mappings(launch, flags):
    """Deflection counts travel in the link slots across patch edges (stamped halves), and
    held ops and delayed injections across launch boundaries, exactly."""
    p = W.config0().with_(width=20, height=13, seed=8, bg_thr=W.thr(0.3), op_thr=W.thr(0.5), flags=flags)
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800])


@pytest.mark.parametrize("flags", FLAG_SETS, ids=IDS)
def test_variants_config2_full_size_prefix(flags):
    """208x208 (43,264 tiles) in the default launch configuration."""
    assert_same_run(W.config2(0.1).with_(flags=flags), 100, step_sizes=[40, 60])


@pytest.mark.parametrize("flags", [DELAY, AGE, HUM, AGE | DELAY, AGE | HUM | DELAY],
                         ids=["delay", "age", "hum", "age_delay", "all"])
@pytest.mark.parametrize("reply_flits", [1, 3])
def test_fast_kernel_variants_on_both_kernels(reply_flits, flags):
    """The variants on the one-tile-per-thread kernel equal the general kernel and the oracle,
    with single- and multi-flit replies, across launch boundaries."""
    p = W.config0().with_(width=24, height=9, seed=55 + reply_flits + flags, bg_thr=W.thr(0.2), op_thr=W.thr(0.6),
                          flags=flags, reply_flits=reply_flits)
    a = gpu_sim(p)
    b = gpu_sim(p, generic=True)
    assert (a.step(777, digests=True) == b.step(777, digests=True)).all()
    assert (a.dump() == b.dump()).all()
    assert_same_run(p, 1200, step_sizes=[500, 700])


@pytest.mark.parametrize("flags", [0, AGE | HUM | DELAY], ids=["base", "all"])
@pytest.mark.parametrize("D", [2, 3, 8])
def test_fast_kernel_router_delay_on_both_kernels(D, flags):
    """Router pipelines on the one-tile-per-thread kernel equal the general kernel and the
    oracle, alone and with every other flag, across launch boundaries."""
    p = W.config0().with_(width=17, height=11, seed=70 + D + flags, bg_thr=W.thr(0.25), op_thr=W.thr(0.5),
                          flags=flags, router_delay=D, reply_flits=2)
    a = gpu_sim(p)
    b = gpu_sim(p, generic=True)
    assert (a.step(555, digests=True) == b.step(555, digests=True)).all()
    assert (a.dump() == b.dump()).all()
    assert_same_run(p, 900, launch=(17, 4, 128, 0), step_sizes=[400, 500])


def test_fast_kernel_variants_batch():
    """One launch of the one-tile-per-thread kernel over base chips and chips with variants
    (some with multi-flit replies): each equals its own oracle run."""
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=5000 + i, bg_thr=W.thr(0.15), flags=f, reply_flits=r)
              for i, (s, f, r) in enumerate([(8, 0, 1), (16, DELAY, 1), (8, AGE, 4), (12, 0, 2), (16, AGE | DELAY, 2),
                                             (12, HUM, 1), (8, AGE | HUM | DELAY, 3)])]
    params += [W.config1().with_(width=10, height=10, seed=5100, bg_thr=W.thr(0.2), router_delay=2),
               W.config1().with_(width=9, height=12, seed=5101, bg_thr=W.thr(0.2), router_delay=5, flags=AGE | HUM)]
    sims = [gpu_sim(p, launch=(p.width, 256 // p.width, 256, 0)) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123, 200, 280, 333, 310, 290])
    for p, s, n in zip(params, sims, [300, 250, 300, 123, 200, 280, 333, 310, 290]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} flags {p.flags} reply_flits {p.reply_flits}"


def test_variants_refuse_the_base_kernel():
    """Asking for the one-tile-per-thread kernel keeps a chip with the directory on the
    general kernel."""
    p = W.config0().with_(width=8, height=8, seed=4, bg_thr=W.thr(0.3), flags=AGE | HUM | W.LSPD, router_delay=2)
    a = gpu_sim(p)
    a.set_kernel(False)
    b = gpu_sim(p, generic=True)
    assert (a.step(600, digests=True) == b.step(600, digests=True)).all()


@pytest.mark.parametrize("flags", FLAG_SETS, ids=IDS)
def test_variants_checkpoint_and_drain_on_gpu(flags):
    p = W.config0().with_(width=6, height=6, seed=31 + flags, bg_thr=W.thr(0.25), op_thr=W.thr(0.5), flags=flags,
                          reply_flits=2, l1_sets=8, shared_lines=512)
    a = gpu_sim(p)
    da = a.step(1000, digests=True)
    b = gpu_sim(p)
    b.step(451)
    snap = b.dump()
    if flags & AGE:
        assert (split_dump(snap, p)["ages"] > 0).any()
    c = gpu_sim(p)
    c.load(snap)
    assert (c.step(549, digests=True) == da[451:]).all()
    o = O.OracleSim(p)
    o.load(snap)
    o.step(549)
    assert (c.dump() == o.dump()).all()
    for s in (a, o):
        s.set_rates(0, 0)
        s.step(3000)
    assert (a.dump() == o.dump()).all()
    assert o.quiescent()
    st = a.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]] == st[STAT["reply_sent"]] == st[STAT["reply_received"]]
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]]


def test_variant_dump_is_refused_by_another_variant():
    p = W.config0().with_(width=4, height=4, flags=AGE)
    a = gpu_sim(p)
    a.step(300)
    other = gpu_sim(p.with_(flags=HUM))
    with pytest.raises(Exception):
        other.load(a.dump())


def test_variants_batch_with_base_chips():
    """One launch over chips of different variants and base-model chips: each equals its
    own oracle run (the whole batch runs on the general kernel)."""
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=4000 + i, bg_thr=W.thr(0.15), flags=f)
              for i, (s, f) in enumerate([(8, 0), (16, AGE), (8, HUM), (24, DELAY), (16, AGE | HUM | DELAY)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123, 200])
    for p, s, n in zip(params, sims, [300, 250, 300, 123, 200]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} flags {p.flags}"


# ---- router delay -------------------------------------------------------------------------------
@pytest.mark.parametrize("D", [2, 3, 8])
def test_router_delay_config0_full_run(D):
    assert_same_run(W.config0().with_(router_delay=D, op_thr=W.thr(0.5)), 6000, step_sizes=[1, 999, 5000])


@pytest.mark.parametrize("D,flags", [(2, 0), (3, AGE), (4, AGE | HUM | DELAY)])
@pytest.mark.parametrize("w,h", [(1, 7), (5, 5), (13, 7)])
def test_router_delay_small_shapes(w, h, D, flags):
    p = W.config0().with_(width=w, height=h, seed=w * 100 + h + D, bg_thr=W.thr(0.25), op_thr=W.thr(0.6),
                          l1_sets=8, shared_lines=256, flags=flags, router_delay=D, reply_flits=2)
    assert_same_run(p, 2500)


@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (20, 1, 64, 0), (5, 5, 64, 37), (20, 13, 64, 0)])
def test_router_delay_patch_mappings(launch):
    """Pipelines are tile-owned: any patch mapping and chunk length gives the same run."""
    p = W.config0().with_(width=20, height=13, seed=9, bg_thr=W.thr(0.3), op_thr=W.thr(0.5), router_delay=3,
                          flags=AGE)
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800])


def test_router_delay_config2_full_size_prefix():
    assert_same_run(W.config2(0.1).with_(router_delay=2), 100, step_sizes=[40, 60])


@pytest.mark.parametrize("D", [2, 5])
def test_router_delay_checkpoint_and_drain_on_gpu(D):
    p = W.config0().with_(width=6, height=6, seed=41 + D, bg_thr=W.thr(0.25), op_thr=W.thr(0.5), router_delay=D,
                          flags=AGE)
    a = gpu_sim(p)
    da = a.step(1000, digests=True)
    b = gpu_sim(p)
    b.step(433)
    snap = b.dump()
    assert (split_dump(snap, p)["pipe"][..., 0] >= 0).any()
    c = gpu_sim(p)
    c.load(snap)
    assert (c.step(567, digests=True) == da[433:]).all()
    o = O.OracleSim(p)
    o.load(snap)
    o.step(567)
    assert (c.dump() == o.dump()).all()
    for s in (a, o):
        s.set_rates(0, 0)
        s.step(3000)
    assert (a.dump() == o.dump()).all()
    assert o.quiescent()
    with pytest.raises(Exception):
        gpu_sim(p.with_(router_delay=D + 1)).load(snap)


def test_router_delay_batch_mixed():
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=5000 + i, bg_thr=W.thr(0.15), router_delay=d)
              for i, (s, d) in enumerate([(8, 1), (16, 2), (8, 5), (24, 3)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123])
    for p, s, n in zip(params, sims, [300, 250, 300, 123]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} router_delay {p.router_delay}"


def test_serving_mixed_model_options_equal_solo_runs():
    """Jobs with different model options share the scheduler's batched launches; each job's
    statistics equal those of the oracle run of the same job."""
    from paper_1508_03235_amd import serve
    import random
    rng = random.Random(5)
    opts = [dict(), dict(flags=AGE), dict(flags=HUM | DELAY, reply_flits=4), dict(router_delay=3),
            dict(flags=W.LSPD, mig_threshold=2, private_lines=64), dict(flags=W.LSPD | W.LSPD_CENTRAL, private_lines=64)]
    jobs = []
    for i, o in enumerate(opts * 2):
        side = rng.choice([8, 12, 16])
        p = W.config1().with_(width=side, height=side, seed=9000 + i, bg_thr=W.thr(0.1), l2_sets=16, **o)
        jobs.append(W.Job(i, 0.001 * i, rng.choice([300, 500, 700]), p))
    srv = serve.Server(serve.GpuBackend(), budget_bytes=8 << 30, tick_cycles=200)
    rep = srv.run(jobs)
    for r, j in zip(rep.results, jobs):
        assert r.error is None, r.error
        o = O.OracleSim(j.params)
        o.step(j.cycles)
        assert (r.stats == o.stats()).all(), f"job {j.index} {j.params.flags}"


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "general"])
def test_deflection_count_limit_on_gpu(generic):
    """A flit one below the 16-bit deflection limit leaves with the limit, as in the oracle; at
    the limit one more deflection stops the run with an invariant failure on both kernels."""
    from paper_1508_03235_amd import nocsim
    from tests.test_oracle_variants import contended_pair_at_centre
    p, snap = contended_pair_at_centre(0xFFFE)
    g = gpu_sim(p, generic=generic)
    g.load(snap)
    g.step(1)
    o = O.OracleSim(p)
    o.load(snap)
    o.step(1)
    assert (g.dump() == o.dump()).all()
    p, snap = contended_pair_at_centre(0xFFFF)
    g = gpu_sim(p, generic=generic)
    g.load(snap)
    with pytest.raises(nocsim.SimError, match="EINVARIANT"):
        g.step(1)


def test_fast_kernel_every_option_full_size():
    """208x208 in the default launch configuration with every option the one-tile-per-thread
    kernel carries: deflection-count priority, hit under miss, the injection register, a
    router delay of 3 and 4-flit replies, against the oracle cycle by cycle."""
    p = W.config2(0.1).with_(flags=AGE | HUM | DELAY, router_delay=3, reply_flits=4)
    assert_same_run(p, 90, step_sizes=[35, 55])
