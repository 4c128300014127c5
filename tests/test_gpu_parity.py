"""Parity of the HIP path (through the C ABI) with the serial oracle.

Bar: bit-exact.  Every per-cycle state digest and the final canonical dump (link slots,
core words, queue nodes, every L1/L2 tag in LRU order, all statistics) must be identical.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import STAT, load_golden, run_flit_trace, run_op_trace, split_dump

pytestmark = pytest.mark.gpu


def gpu_sim(p, launch=None, generic=False):
    from paper_1508_03235_amd import nocsim
    s = nocsim.Sim(p)
    if launch:
        s.set_launch(*launch)
    if generic:
        s.set_kernel(True)
    return s


def assert_same_run(p, cycles, launch=None, step_sizes=None, generic=False):
    g = gpu_sim(p, launch, generic)
    o = O.OracleSim(p)
    steps = step_sizes or [cycles]
    for n in steps:
        dg = g.step(n, digests=True)
        do = o.step(n, digests=True)
        bad = np.nonzero(dg != do)[0]
        assert len(bad) == 0, f"{p.width}x{p.height} launch={launch}: digest differs at cycle {g.cycle - n + bad[0]}"
    a, b = g.dump(), o.dump()
    if not (a == b).all():
        da, db = split_dump(a, p), split_dump(b, p)
        for k in ("links", "core", "l1", "l2", "stats", "ages", "pipe", "loc", "l2rec"):
            if not np.array_equal(da[k], db[k]):
                idx = np.argwhere(da[k] != db[k])[:5]
                raise AssertionError(f"dump section {k} differs at {idx.tolist()}")
    return g, o


GOLD = load_golden("hand_traces.json")


@pytest.mark.parametrize("tr", GOLD["flit_traces"], ids=lambda t: t["name"])
def test_gpu_hand_flit_trace(tr):
    run_flit_trace(gpu_sim, tr)


@pytest.mark.parametrize("tr", GOLD["op_traces"], ids=lambda t: t["name"])
def test_gpu_hand_op_trace(tr):
    run_op_trace(gpu_sim, tr)


def test_config0_full_run():
    """4x4, 10,000 cycles, background 0.05 + Zipf(0.8) cache traffic, seed 1."""
    assert_same_run(W.config0(), 10_000, step_sizes=[1, 999, 4000, 5000])


@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (9, 1), (2, 3), (5, 5), (13, 7)])
def test_small_shapes(w, h):
    p = W.config0().with_(width=w, height=h, seed=w * 100 + h, bg_thr=W.thr(0.2) if w * h > 1 else 0,
                          op_thr=W.thr(0.5))
    assert_same_run(p, 3000)


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (3, 5, 64, 0), (7, 2, 64, 0), (20, 1, 64, 0), (1, 13, 64, 0),
                                    (5, 5, 64, 37), (20, 13, 64, 0), (16, 8, 128, 0)])
def test_patch_mappings_are_exact(launch, generic):
    """The chip cut into patches (edges exchanged through stamped slots) gives the same run
    as the oracle for patch shapes that do and do not divide the mesh, odd chunk lengths,
    one tile per thread (fast kernel) and several tiles per thread (general kernel)."""
    p = W.config0().with_(width=20, height=13, seed=5, bg_thr=W.thr(0.15), op_thr=W.thr(0.5))
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800], generic=generic)


def test_config1_prefix():
    """64x64, the cache-only model (30% shared Zipf(0.9) over 2^24 lines, 70% private)."""
    assert_same_run(W.config1(), 1500, step_sizes=[500, 1000])


@pytest.mark.parametrize("rate", [0.01, 0.3])
def test_config2_full_size_prefix(rate):
    """208x208 (43,264 tiles) in the launch configuration the benchmark times: a prefix of
    the run, every cycle compared."""
    assert_same_run(W.config2(rate), 120, step_sizes=[50, 70])


def test_config2_general_kernel_prefix():
    assert_same_run(W.config2(0.1), 60, generic=True)


def test_repeatable_and_mapping_independent():
    p = W.config0().with_(width=16, height=16, seed=3, bg_thr=W.thr(0.1), op_thr=W.thr(0.4))
    runs = []
    for launch, generic in [(None, False), ((4, 4, 64, 0), False), ((16, 1, 64, 0), False), ((8, 8, 64, 100), False),
                            ((4, 4, 64, 0), True), ((16, 16, 64, 0), True)]:
        g = gpu_sim(p, launch, generic)
        runs.append(g.step(800, digests=True))
    for r in runs[1:]:
        assert (r == runs[0]).all()


def test_checkpoint_resume_on_gpu():
    p = W.config0().with_(width=8, height=8, seed=11, bg_thr=W.thr(0.1))
    a = gpu_sim(p)
    da = a.step(1000, digests=True)
    b = gpu_sim(p)
    b.step(400)
    snap = b.dump()
    c = gpu_sim(p)
    c.load(snap)
    dc = c.step(600, digests=True)
    assert (dc == da[400:]).all()
    assert (c.dump() == a.dump()).all()


def test_drain_on_gpu_matches_oracle():
    p = W.config0().with_(width=6, height=6, seed=21, bg_thr=W.thr(0.2), op_thr=W.thr(0.5))
    g, o = gpu_sim(p), O.OracleSim(p)
    g.step(1500)
    o.step(1500)
    g.set_rates(0, 0)
    o.set_rates(0, 0)
    g.step(1500)
    o.step(1500)
    assert (g.dump() == o.dump()).all()
    assert o.quiescent()
    st = g.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]] == st[STAT["reply_sent"]] == st[STAT["reply_received"]]


def test_batch_each_chip_matches_its_own_run():
    """Chips of uneven sizes, seeds and rates advanced by one launch equal their oracle runs."""
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=1000 + i, bg_thr=W.thr(r))
              for i, (s, r) in enumerate([(8, 0.01), (16, 0.3), (24, 0.1), (8, 0.2), (32, 0.05)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    cycles = [300, 250, 300, 123, 0]
    b.step(cycles)
    b.step([200, 250, 0, 77, 100])
    for p, s, c0, c1 in zip(params, sims, cycles, [200, 250, 0, 77, 100]):
        o = O.OracleSim(p)
        o.step(c0 + c1)
        assert s.cycle == c0 + c1
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} seed {p.seed}"


def test_batch_split_into_resident_groups():
    """A batch with more workgroups than the device holds at once runs as several launch
    groups; every chip still equals its own oracle run."""
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=32, height=32, seed=2000 + i, bg_thr=W.thr(0.05 + 0.01 * (i % 5)),
                                l2_sets=64, l1_sets=32) for i in range(40)]
    sims = [gpu_sim(p, launch=(4, 4, 64, 0)) for p in params]   # 64 patches per chip, 2,560 in all
    b = nocsim.Batch(sims, block=64)
    b.step([150] * len(sims))
    for i in (0, 17, 39):
        o = O.OracleSim(params[i])
        o.step(150)
        assert (sims[i].dump() == o.dump()).all(), f"chip {i}"


@pytest.mark.parametrize("w,h", [(700, 3), (3, 700), (1, 1500), (300, 17)])
def test_wide_and_tall_chips(w, h):
    """Chips wider than 256 columns (rows cut into three or more strips) and very tall or
    one-column chips."""
    p = W.config0().with_(width=w, height=h, seed=w + 7 * h, bg_thr=W.thr(0.1), op_thr=W.thr(0.3),
                          l1_sets=16, l2_sets=32)
    assert_same_run(p, 150, step_sizes=[60, 90])


@pytest.mark.parametrize("w,h,strips", [(100, 2048, False), (256, 300, True)])
def test_default_mapping_of_tall_chips(w, h, strips):
    """A 256x300 chip's 600 row strips are all resident with four two-wave workgroups per
    compute unit (the narrow build of the one-tile-per-thread kernel); a 100x2048 chip's 2,048
    strips are not, and the default mapping falls back to square-ish patches, about one per
    compute unit."""
    p = W.config0().with_(width=w, height=h, seed=w + h, bg_thr=W.thr(0.1), op_thr=W.thr(0.3),
                          l1_sets=16, l2_sets=32)
    g = gpu_sim(p)
    pw, ph, block, _ = g.get_launch()
    if strips:
        assert (pw, ph, block) == (128, 1, 128)
    else:
        assert -(-w // pw) * -(-h // ph) <= 256 and pw * ph > block
    del g
    assert_same_run(p, 40, step_sizes=[15, 25])


def test_largest_line_numbers():
    """252x256 tiles with 2^14 private lines each: the top private line is 2^30 - 1, the
    largest line the flit format holds."""
    p = W.config1().with_(width=252, height=256, l1_sets=16, l2_sets=16, op_thr=W.thr(0.9), shared_thr=0)
    assert p.shared_lines + p.tiles * p.private_lines == 2**30
    assert_same_run(p, 25)


def test_autotuned_mapping_gives_the_same_run(tmp_path):
    from paper_1508_03235_amd import autotune
    p = W.config1().with_(width=40, height=24, seed=77, bg_thr=W.thr(0.1))
    best = autotune.tune(p, cycles=100, warmup=20, cache_path=str(tmp_path / "tune.json"))
    assert len(best) == 3
    assert autotune.tune(p, cache_path=str(tmp_path / "tune.json")) == best   # cached
    assert_same_run(p, 400, launch=(best[0], best[1], best[2], 0))


# ---- multi-flit reply packets (Sec. 3.6, Table 1) --------------------------------------------

def test_packets_config0_full_run():
    """4x4, 10,000 cycles with 4-flit replies (the paper's remote L2 access)."""
    assert_same_run(W.config0().with_(reply_flits=4), 10_000, step_sizes=[1, 999, 4000, 5000])


@pytest.mark.parametrize("flits", [2, 16])
@pytest.mark.parametrize("w,h", [(1, 7), (5, 5), (13, 7)])
def test_packets_small_shapes(w, h, flits):
    p = W.config0().with_(width=w, height=h, seed=w * 100 + h + flits, bg_thr=W.thr(0.2), op_thr=W.thr(0.5),
                          reply_flits=flits)
    assert_same_run(p, 3000)


@pytest.mark.parametrize("generic", [False, True], ids=["fast", "generic"])
@pytest.mark.parametrize("launch", [(4, 4, 64, 0), (7, 2, 64, 0), (20, 1, 64, 0), (5, 5, 64, 37)])
def test_packets_patch_mappings(launch, generic):
    """Partially sent replies (node words written by the home) and partially received ones
    (a core word) cross patch edges and launch boundaries exactly."""
    p = W.config0().with_(width=20, height=13, seed=6, bg_thr=W.thr(0.15), op_thr=W.thr(0.5), reply_flits=4)
    assert_same_run(p, 1500, launch=launch, step_sizes=[700, 800], generic=generic)


def test_packets_config2_full_size_prefix():
    assert_same_run(W.config2(0.05).with_(reply_flits=4), 120, step_sizes=[50, 70])


def test_packets_checkpoint_and_drain_on_gpu():
    p = W.config0().with_(width=6, height=6, seed=23, bg_thr=W.thr(0.2), op_thr=W.thr(0.5), reply_flits=4)
    a = gpu_sim(p)
    da = a.step(1000, digests=True)
    b = gpu_sim(p)
    b.step(437)
    c = gpu_sim(p)
    c.load(b.dump())
    assert (c.step(563, digests=True) == da[437:]).all()
    o = O.OracleSim(p)
    o.step(1000)
    for s in (a, o):
        s.set_rates(0, 0)
        s.step(3000)
    assert (a.dump() == o.dump()).all()
    assert o.quiescent()
    st = a.stats()
    assert st[STAT["inj_reply"]] == st[STAT["ej_reply"]] == 4 * st[STAT["reply_sent"]]
    assert st[STAT["reply_sent"]] == st[STAT["reply_received"]] == st[STAT["req_made"]]


def test_packets_batch_of_mixed_reply_sizes():
    """One launch over chips with 1-, 2-, 4- and 16-flit replies equals their own runs."""
    from paper_1508_03235_amd import nocsim
    params = [W.config1().with_(width=s, height=s, seed=3000 + i, bg_thr=W.thr(0.1), reply_flits=f)
              for i, (s, f) in enumerate([(8, 1), (16, 4), (8, 16), (24, 2), (16, 1)])]
    sims = [gpu_sim(p) for p in params]
    b = nocsim.Batch(sims)
    b.step([300, 250, 300, 123, 200])
    for p, s, n in zip(params, sims, [300, 250, 300, 123, 200]):
        o = O.OracleSim(p)
        o.step(n)
        assert (s.dump() == o.dump()).all(), f"chip {p.width}x{p.height} reply_flits {p.reply_flits}"
