"""Parity of block migration and redirection (Sec. 3.3) on the GPU with the serial oracle.

A migrating chip runs on the one-tile-per-thread kernel by default; the main cases run on both
that kernel and the general one."""
from functools import partial

import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import CORE, STAT, split_dump
from tests.test_gpu_parity import assert_same_run, gpu_sim
from tests import test_oracle_migration as OM

pytestmark = pytest.mark.gpu

LSPD, CENTRAL = W.LSPD, W.LSPD_CENTRAL


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_gpu_hand_trace_migration_then_redirection(generic):
    """The oracle's hand trace on the GPU: the block migrates (31) and a request that reaches
    the source after the arrival notice is redirected (17)."""
    OM.test_hand_trace_migration_then_redirection(make_sim=partial(gpu_sim, generic=generic))


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_gpu_hand_trace_source_serves_during_transit(generic):
    """A request that reaches the source while the block is on its way is served there (14)."""
    OM.test_hand_trace_source_serves_during_transit(make_sim=partial(gpu_sim, generic=generic))


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_gpu_hand_trace_source_evicts_the_block_on_its_way(generic):
    """The source's one-way slice drops the block while it is on its way: no eviction notice."""
    OM.test_hand_trace_source_evicts_the_block_on_its_way(make_sim=partial(gpu_sim, generic=generic))


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_gpu_migration_races_under_pressure(seed, generic):
    """The oracle's high-pressure migration runs (late arrival notices, sources evicting blocks
    on their way, blocks moving on before the notice): every digest and the state after a
    drain equal the oracle's."""
    import random
    rng = random.Random(500 + seed)
    w, h = [(3, 3), (4, 4), (3, 2), (5, 3)][seed % 4]
    p = OM._params(rng, w, h, LSPD | (CENTRAL if seed % 2 else 0), 1, op_thr=W.thr(0.9), shared_thr=W.thr(0.95),
                   shared_lines=6 + seed, private_lines=2, bg_thr=0, reply_flits=1 + seed % 3, mem_lat=5,
                   l2_sets=1, l2_ways=1 + seed % 2, l1_sets=1)
    g, o = assert_same_run(p, 2000, step_sizes=[1, 999, 1000], generic=generic)
    for s in (g, o):
        s.set_rates(0, 0)
        s.step(2000)
    assert o.quiescent() and (g.dump() == o.dump()).all()


@pytest.mark.parametrize("mig,pattern,moved", OM.MAJORITY_CASES + [(3, [8, 0, 4], 0), (16, [8] * 9, 1),
                                                                  (16, [8] * 8, 0)])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_gpu_majority_of_the_last_n_accesses(mig, pattern, moved, generic):
    g = OM.remote_reads(mig, pattern, make_sim=partial(gpu_sim, generic=generic))
    o = OM.remote_reads(mig, pattern)
    assert g.stat("migrations") == o.stat("migrations") == moved
    assert (g.dump() == o.dump()).all()   # tags, histories, forwarding words, location array


@pytest.mark.parametrize("thr", [1, 2, 4])
@pytest.mark.parametrize("flags", [LSPD, LSPD | CENTRAL], ids=["interleaved", "central"])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_migration_config0_run(flags, thr, generic):
    p = W.config0().with_(flags=flags, mig_threshold=thr, op_thr=W.thr(0.5), l1_sets=2, l1_ways=1, l2_sets=8,
                          l2_ways=2, shared_lines=256, reply_flits=4)
    assert_same_run(p, 6000, step_sizes=[1, 999, 5000], generic=generic)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (5, 5), (13, 7)])
@pytest.mark.parametrize("flags", [LSPD, LSPD | W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY],
                         ids=["lspd", "with_variants"])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_migration_small_shapes(w, h, flags, generic):
    p = W.config1().with_(width=w, height=h, seed=w * 100 + h + flags, bg_thr=W.thr(0.1) if w * h > 1 else 0,
                          op_thr=W.thr(0.6), l1_sets=2, l1_ways=1, l2_sets=8, l2_ways=2, shared_lines=256,
                          private_lines=32, flags=flags, mig_threshold=1, reply_flits=2, router_delay=2)
    assert_same_run(p, 3000, generic=generic)


@pytest.mark.parametrize("w,h,launch", [(13, 7, None), (20, 13, (5, 5, 64, 0)), (20, 13, (20, 1, 64, 37))])
@pytest.mark.parametrize("mig", [1, 2])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_migration_ways48_single_flit(w, h, launch, mig, generic):
    """4-way L1, 8-way slices of 4 sets, single-flit replies, no variants: the migration build
    compiled for those way counts; with a history of one, blocks move, are evicted and are
    redirected all the time."""
    p = W.config1().with_(width=w, height=h, seed=w * 37 + h + mig, bg_thr=W.thr(0.1), op_thr=W.thr(0.6), l1_sets=8,
                          l2_sets=4, shared_lines=256, shared_thr=W.thr(0.8), private_lines=32, flags=LSPD,
                          mig_threshold=mig)
    g, o = assert_same_run(p, 3000, launch=launch, step_sizes=[1000, 2000], generic=generic)
    if mig == 1:  # (a remote majority of the last two accesses is rare under this sharing)
        assert g.stat("migrations") > 0 and g.stat("redirects") > 0


@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (7, 2, 64, 0), (20, 1, 64, 0), (5, 5, 64, 37), (20, 13, 64, 0)])
@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_migration_patch_mappings(launch, generic):
    p = W.config1().with_(width=20, height=13, seed=12, bg_thr=W.thr(0.1), op_thr=W.thr(0.5), l1_sets=2, l1_ways=1,
                          l2_sets=8, l2_ways=2, shared_lines=512, private_lines=32, flags=LSPD, mig_threshold=2)
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800], generic=generic)


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
def test_migration_208x208_prefix(generic):
    p = W.config2(0.05).with_(flags=LSPD, private_lines=2**10, mig_threshold=2)
    assert_same_run(p, 80, step_sizes=[30, 50], generic=generic)


def test_migration_checkpoint_mid_claim_and_drain():
    p = W.config1().with_(width=6, height=6, seed=61, bg_thr=W.thr(0.1), op_thr=W.thr(0.5), l1_sets=2, l1_ways=1,
                          l2_sets=8, l2_ways=2, shared_lines=128, private_lines=16, flags=LSPD, mig_threshold=1,
                          reply_flits=4)
    b = gpu_sim(p)
    for _ in range(3000):
        b.step(1)
        core = split_dump(b.dump(), p)["core"]
        if ((core[:, CORE["state"]] == 3) & (core[:, CORE["claim"]] >= 0)).any():
            break
    else:
        raise AssertionError("no pending claim seen")
    k = b.cycle
    snap = b.dump()
    a = gpu_sim(p)
    da = a.step(k + 700, digests=True)
    c = gpu_sim(p)
    c.load(snap)
    assert (c.step(700, digests=True) == da[k:]).all()
    o = O.OracleSim(p)
    o.load(snap)
    o.step(700)
    assert (c.dump() == o.dump()).all()
    for s in (a, o):
        s.set_rates(0, 0)
        s.step(3000)
    assert (a.dump() == o.dump()).all()
    assert o.quiescent()
    assert a.stats()[STAT["migrations"]] > 0


def test_migration_batch_with_other_chips():
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=7000 + i, bg_thr=W.thr(0.1), l1_sets=2, l1_ways=1,
                                l2_sets=16, shared_lines=2048, private_lines=64, flags=f, mig_threshold=m)
              for i, (s, f, m) in enumerate([(8, 0, 0), (16, LSPD, 2), (8, LSPD | CENTRAL, 1), (24, LSPD, 0)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123])
    for p, s, n in zip(params, sims, [300, 250, 300, 123]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} flags {p.flags} mig {p.mig_threshold}"


def test_full_size_long_prefix_every_option():
    """208x208 with the directory, migration on every remote access, multi-flit replies, the
    three variants and a router delay: 400 cycles, every digest equal to the oracle's, then the
    whole canonical state (location array and way records included)."""
    p = W.config2(0.1).with_(flags=LSPD | W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY, private_lines=2**10,
                             mig_threshold=1, reply_flits=4, router_delay=2, l1_sets=4, l1_ways=1)
    assert_same_run(p, 400, step_sizes=[150, 250])
