"""Parity of the LSPD directory model (SimParams.flags LSPD) on the GPU with the serial oracle.

Bit-exact, as for the base model: per-cycle digests (which carry each directory tile's
checksum of its entries) and the final canonical dump, location array included.  Without
migration a chip runs on the one-tile-per-thread kernel by default; the main cases run on both
that kernel and the general one.
"""
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import STAT, split_dump
from tests.test_gpu_parity import assert_same_run, gpu_sim
from tests.test_oracle_lspd import M, _quiet, _run_ops

pytestmark = pytest.mark.gpu

LSPD, CENTRAL = W.LSPD, W.LSPD_CENTRAL
MODES = [LSPD, LSPD | CENTRAL]
IDS = ["interleaved", "central"]


def test_gpu_hand_traces():
    """The oracle's hand traces, on the GPU: cold (M + 4), remote (11), local directory (5),
    L1 hit (0); and the trap after an eviction (1 + M, M + 16)."""
    sim = gpu_sim(_quiet(2, 2))
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    assert _run_ops(sim, [(sim.cycle + 2, 3, 5)]) == {0: 11}
    assert _run_ops(sim, [(sim.cycle + 2, 1, 5)]) == {0: 5}
    assert _run_ops(sim, [(sim.cycle + 2, 0, 5)]) == {0: 0}
    p = _quiet(2, 2, l2_sets=1, l2_ways=1)
    sim = gpu_sim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    a = sim.cycle + 3
    F = a + 1 + M
    assert _run_ops(sim, [(a, 0, 8), (F - 5, 2, 5)]) == {0: 1 + M, 1: M + 16}
    assert sim.stats()[STAT["trap"]] == 1


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
@pytest.mark.parametrize("flags", MODES, ids=IDS)
def test_lspd_config0_full_run(flags, generic):
    """4x4, 10,000 cycles of config 0 with the directory (small slices, so blocks are evicted
    and entries go stale)."""
    p = W.config0().with_(flags=flags, op_thr=W.thr(0.5), l2_sets=16, l2_ways=2, shared_lines=2048, reply_flits=4)
    assert_same_run(p, 10_000, step_sizes=[1, 999, 4000, 5000], generic=generic)


@pytest.mark.parametrize("flags", MODES + [LSPD | W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY],
                         ids=IDS + ["with_variants"])
@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (5, 5), (13, 7)])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_lspd_small_shapes(w, h, flags, generic):
    p = W.config1().with_(width=w, height=h, seed=w * 100 + h + flags, bg_thr=W.thr(0.1) if w * h > 1 else 0,
                          op_thr=W.thr(0.6), l1_sets=8, l2_sets=8, l2_ways=2, shared_lines=512, private_lines=64,
                          flags=flags, reply_flits=2)
    assert_same_run(p, 3000, generic=generic)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("flags", MODES + [LSPD | W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY],
                         ids=IDS + ["with_variants"])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_lspd_router_delay(D, flags, generic):
    """The directory with a router delay of D cycles per hop and 3-flit replies."""
    p = W.config1().with_(width=9, height=6, seed=77 + D, bg_thr=W.thr(0.1), op_thr=W.thr(0.6), l1_sets=8, l2_sets=8,
                          l2_ways=2, shared_lines=512, private_lines=64, flags=flags, reply_flits=3, router_delay=D)
    assert_same_run(p, 2500, step_sizes=[1000, 1500], generic=generic)


@pytest.mark.parametrize("w,h,launch", [(13, 7, None), (20, 13, (5, 5, 64, 0)), (20, 13, (20, 1, 64, 37))])
@pytest.mark.parametrize("flags", MODES, ids=IDS)
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_lspd_ways48_single_flit(w, h, launch, flags, generic):
    """4-way L1, 8-way slices of 4 sets (blocks are evicted from the slices all the time),
    single-flit replies, no variants: the directory build compiled for those way counts."""
    p = W.config1().with_(width=w, height=h, seed=w * 31 + h, bg_thr=W.thr(0.1), op_thr=W.thr(0.5), l1_sets=8, l2_sets=4,
                          shared_lines=2048, private_lines=64, flags=flags)
    assert_same_run(p, 3000, launch=launch, step_sizes=[1000, 2000], generic=generic)


@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (7, 2, 64, 0), (20, 1, 64, 0), (5, 5, 64, 37), (20, 13, 64, 0)])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_lspd_patch_mappings(launch, generic):
    """Directory accesses, answers, traps and eviction notices cross patch edges and launch
    boundaries exactly; entries are only touched by their directory tile."""
    p = W.config1().with_(width=20, height=13, seed=10, bg_thr=W.thr(0.1), op_thr=W.thr(0.5), l2_sets=8, l2_ways=2,
                          shared_lines=1024, private_lines=64, flags=LSPD)
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800], generic=generic)


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
@pytest.mark.parametrize("flags", MODES, ids=IDS)
def test_lspd_208x208_prefix(flags, generic):
    """The 208x208 chip (43,264 tiles) with the directory, 2^10 private lines per tile."""
    p = W.config2(0.05).with_(flags=flags, private_lines=2**10)
    assert_same_run(p, 80, step_sizes=[30, 50], generic=generic)


@pytest.mark.parametrize("mig", [0, 1], ids=["directory", "migration"])
def test_lspd_208x208_past_memory_latency_timed_build(mig):
    """The 208x208 chip with the directory (and with migration at a history of 1) for 1,200
    cycles, past the 200-cycle memory latency, on the build the benchmark times (no digests):
    the whole state, location array and histories included, equals the oracle's."""
    p = W.config2(0.05).with_(flags=LSPD, mig_threshold=mig, private_lines=2**10)
    g = gpu_sim(p)
    g.step(1200)
    o = O.OracleSim(p)
    o.step(1200)
    assert (g.dump() == o.dump()).all()
    assert g.stat("dir_nack") > 0 and g.stat("l2_hit") > 0


@pytest.mark.parametrize("flags", MODES, ids=IDS)
def test_lspd_checkpoint_and_drain_on_gpu(flags):
    p = W.config1().with_(width=6, height=6, seed=51, bg_thr=W.thr(0.1), op_thr=W.thr(0.5), l2_sets=8, l2_ways=2,
                          shared_lines=512, private_lines=32, flags=flags, reply_flits=4)
    a = gpu_sim(p)
    da = a.step(1200, digests=True)
    b = gpu_sim(p)
    b.step(555)
    snap = b.dump()
    c = gpu_sim(p)
    c.load(snap)
    assert (c.step(645, digests=True) == da[555:]).all()
    o = O.OracleSim(p)
    o.load(snap)
    o.step(645)
    assert (c.dump() == o.dump()).all()
    for s in (a, o):
        s.set_rates(0, 0)
        s.step(3000)
    assert (a.dump() == o.dump()).all()
    assert o.quiescent()
    st = a.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]]
    assert st[STAT["dir_access"]] == st[STAT["l2_miss"]] + st[STAT["trap"]]
    with pytest.raises(Exception):
        gpu_sim(p.with_(flags=flags ^ CENTRAL)).load(snap)


def test_lspd_batch_with_other_chips():
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=6000 + i, bg_thr=W.thr(0.1), l2_sets=16, shared_lines=4096,
                                private_lines=128, flags=f)
              for i, (s, f) in enumerate([(8, 0), (16, LSPD), (8, LSPD | CENTRAL), (24, LSPD | W.AGE_DEFLECT)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123])
    for p, s, n in zip(params, sims, [300, 250, 300, 123]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} flags {p.flags}"
