"""Pins of the oracle's LSPD directory model (SimParams.flags LSPD, LSPD_CENTRAL), on the CPU.

The paper's L2 (Sec. 3.2, Sec. 3.4, Sec. 6.2.2, Table 1): a block lives in one slice at a time
(local placement), a location array keyed by line names it, and an L1 miss goes local slice ->
directory access -> owner (remote access) or memory.  Checked here against: latencies of hand
traces worked out from the message sequence, the reduction to the static-home model on a 1x1
chip, the one-copy rule and requester accounting every cycle, the exact equality of directory
and slice contents after a drain, the counting identities of the paper's statistics, and an
independent recomputation of each directory tile's checksum.
"""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import CORE, STAT, quiet_params, split_dump

LSPD, CENTRAL = W.LSPD, W.LSPD_CENTRAL
M = 20  # memory latency of the hand traces


def _run_ops(sim, plan, max_cycles=3000):
    """plan: list of (cycle, tile, line); each op is forced so that it issues in that cycle.
    Returns {index: latency} read from the per-op completion (ops on distinct tiles)."""
    pending = sorted(enumerate(plan), key=lambda x: x[1][0])
    done, lat = {}, {}
    busy = {}
    oracle = isinstance(sim, O.OracleSim)
    for _ in range(max_cycles):
        c = sim.cycle
        while pending and pending[0][1][0] == c:
            i, (_, tile, line) = pending.pop(0)
            sim.force_op(tile, line)
            busy[tile] = (i, c)
        if oracle:
            sim.step(1, check=True)   # the oracle also checks its invariants every cycle
        else:
            sim.step(1)
        core = split_dump(sim.dump(), sim.params)["core"]
        for tile, (i, c0) in list(busy.items()):
            if core[tile, CORE["state"]] == 0 and core[tile, CORE["force_line"]] < 0 and i not in done:
                # idle again: the op completed in the cycle just run
                done[i] = True
                lat[i] = sim.cycle - 1 - c0
                del busy[tile]
        if not pending and not busy:
            return lat
    raise AssertionError("ops did not finish")


def _quiet(w, h, **kw):
    base = dict(l1_lat=1, mem_lat=M, flags=LSPD)
    base.update(kw)
    return quiet_params(w, h, **base)


def test_hand_trace_cold_remote_local_and_hit():
    """2x2, line 5 (directory slice 5 mod 4 = 1).  Tile 0 cold: L1 miss (1), directory access
    over 1 hop (1), lookup the next cycle (1), negative reply over 1 hop (1), memory (M), filled
    into slice 0 and L1 in the cycle it arrives: M + 4.  Tile 3: L1 miss (1), access to the
    directory 1 hop away (1), lookup (1), reply naming tile 0 (1), remote access 2 hops after
    one cycle (1 + 2), lookup at the owner (1), the block back over 2 hops (2), fill the next
    cycle (1): 11.  Tile 1 keeps line 5's entry itself: L1 miss (1), the request to tile 0 at
    once (1 hop: 1), lookup (1), reply (1), fill (1): 5.  Tile 0 again: an L1 hit, 0."""
    p = _quiet(2, 2)
    sim = O.OracleSim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    c = sim.cycle + 2
    assert _run_ops(sim, [(c, 3, 5)]) == {0: 11}
    c = sim.cycle + 2
    assert _run_ops(sim, [(c, 1, 5)]) == {0: 5}
    c = sim.cycle + 2
    assert _run_ops(sim, [(c, 0, 5)]) == {0: 0}
    st = sim.stats()
    assert st[STAT["dir_access"]] == 3 and st[STAT["dir_nack"]] == 1 and st[STAT["trap"]] == 0
    assert st[STAT["req_made"]] == st[STAT["reply_sent"]] == 2
    d = split_dump(sim.dump(), p)
    assert d["loc"][5] == 0
    assert 5 in d["l2"][0].ravel() and 5 not in d["l2"][1:].ravel()


def test_hand_trace_trap_after_eviction():
    """A one-way slice at tile 0 holds line 5.  Tile 0 then reads line 8, whose entry it keeps
    itself: negative reply at once, the block arrives at F = a + 1 + M and evicts line 5, whose
    eviction notice reaches the directory (tile 1) at F + 1 and is applied at F + 2.  Tile 2
    asks for line 5 at b = F - 5: its directory access is answered at F - 1 with the stale owner
    0; its remote access reaches tile 0 at F + 3 and traps at F + 4; the trap reaches tile 2 at
    F + 5, it asks again at F + 6, the directory (cleared) answers no at F + 9, the answer
    arrives at F + 11 and the block M cycles later: latency M + 16, one trap."""
    p = _quiet(2, 2, l2_sets=1, l2_ways=1)
    sim = O.OracleSim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    a = sim.cycle + 3
    F = a + 1 + M
    lat = _run_ops(sim, [(a, 0, 8), (F - 5, 2, 5)])
    assert lat == {0: 1 + M, 1: M + 16}
    st = sim.stats()
    assert st[STAT["trap"]] == 1 and st[STAT["dir_evict"]] == 1 and st[STAT["dir_nack"]] == 3
    d = split_dump(sim.dump(), p)
    assert d["loc"][5] == 2 and d["loc"][8] == 0


@pytest.mark.parametrize("flags", [0, W.HIT_UNDER_MISS])
@pytest.mark.parametrize("s2,w2", [(4, 2), (2, 4), (8, 1)])
def test_one_tile_reduces_to_static_home(flags, s2, w2):
    """On a 1x1 chip every line is local and the directory is the tile itself: the block comes
    from memory after the same delay as with a static home and only the slice fills it, so the
    run equals the static-home run once the last op is done (caches, latencies, counts; only
    the directory counters differ)."""
    base = quiet_params(1, 1, l1_sets=4, l1_ways=2, l2_sets=s2, l2_ways=w2, mem_lat=9, l1_lat=2,
                        op_thr=W.thr(0.5), shared_lines=64, zipf_shared_s=0.7, seed=s2 * 7 + w2, flags=flags)
    a, b = O.OracleSim(base), O.OracleSim(base.with_(flags=flags | LSPD))
    for sim in (a, b):   # run, then let the last op finish (the static home installs a missed
        sim.step(3000, check=True)  # block at lookup, the LSPD slice when it arrives)
        sim.set_rates(0, 0)
        sim.step(100, check=True)
        assert sim.quiescent()
    sa, sb = a.stats(), b.stats()
    for k in STAT:
        if k not in ("dir_access", "dir_nack", "trap", "dir_evict"):
            assert sa[STAT[k]] == sb[STAT[k]], k
    da, db = split_dump(a.dump(), base), split_dump(b.dump(), base.with_(flags=flags | LSPD))
    assert (da["l1"] == db["l1"]).all() and (da["l2"] == db["l2"]).all()
    assert sb[STAT["dir_nack"]] == sb[STAT["l2_miss"]] == sa[STAT["l2_miss"]]


def _params(rng, w, h, flags, **kw):
    base = dict(width=w, height=h, seed=rng.randrange(1 << 40), l1_sets=4, l1_ways=2, l2_sets=4, l2_ways=2,
                l1_lat=rng.choice([1, 2]), mem_lat=rng.choice([5, 30]), op_thr=W.thr(0.5), shared_thr=W.thr(0.5),
                bg_thr=W.thr(0.1), shared_lines=96, private_lines=24, zipf_shared_s=0.8, zipf_private_s=0.8,
                flags=flags)
    base.update(kw)
    return W.SimParams(**base)


def _mix64(z):
    z &= (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & ((1 << 64) - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & ((1 << 64) - 1)
    return z ^ (z >> 31)


def _dir_sums(p, loc):
    N = p.tiles
    central = (p.height // 2) * p.width + p.width // 2
    sums = [0] * N
    for line, owner in enumerate(loc.tolist()):
        if owner >= 0:
            d = central if p.flags & CENTRAL else line % N
            sums[d] = (sums[d] + _mix64((line << 32) | owner)) & ((1 << 64) - 1)
    return sums


FLAG_SETS = [LSPD, LSPD | CENTRAL, LSPD | W.HIT_UNDER_MISS | W.INJECT_DELAY | W.AGE_DEFLECT]


@pytest.mark.parametrize("flags", FLAG_SETS, ids=["interleaved", "central", "with_variants"])
@pytest.mark.parametrize("w,h,flits,D", [(2, 2, 1, 1), (3, 3, 4, 1), (4, 5, 2, 2)])
def test_invariants_drain_and_directory_matches_slices(flags, w, h, flits, D):
    """Every cycle: one copy per block, the directory names the slice that holds it, every
    waiting requester is in exactly one place, conservation; each directory tile's checksum
    equals an independent recomputation from the location array.  After the traffic stops the
    chip drains and the directory equals the slices' contents exactly, and the counters obey
    requests made = received = replies sent + traps, replies sent = received, directory
    accesses = slice misses + traps, negative replies = blocks brought from memory."""
    rng = random.Random(flags + 10 * w + h + D)
    p = _params(rng, w, h, flags, reply_flits=flits, router_delay=D)
    sim = O.OracleSim(p)
    for _ in range(12):
        sim.step(100, check=True)
        d = split_dump(sim.dump(), p)
        sums = _dir_sums(p, d["loc"])
        core = d["core"]
        got = [(int(lo) & 0xFFFFFFFF) | ((int(hi) & 0xFFFFFFFF) << 32)
               for lo, hi in zip(core[:, CORE["dir_sum_lo"]], core[:, CORE["dir_sum_hi"]])]
        assert got == sums
    sim.set_rates(0, 0)
    for _ in range(400):
        if sim.quiescent():
            break
        sim.step(50, check=True)
    assert sim.quiescent()
    st = sim.stats()
    d = split_dump(sim.dump(), p)
    held = {}
    for t in range(p.tiles):
        for line in d["l2"][t].ravel().tolist():
            if line >= 0:
                assert line not in held
                held[line] = t
    loc = d["loc"]
    assert {i: int(o) for i, o in enumerate(loc.tolist()) if o >= 0} == held
    # every remote access arrives and is answered with the block or a trap; the other traps are
    # directory answers naming the asker itself (its own eviction notice still on the way)
    assert st[STAT["req_made"]] == st[STAT["req_received"]] >= st[STAT["reply_sent"]]
    assert st[STAT["trap"]] >= st[STAT["req_received"]] - st[STAT["reply_sent"]]
    assert st[STAT["reply_sent"]] == st[STAT["reply_received"]]
    assert st[STAT["dir_access"]] == st[STAT["l2_miss"]] + st[STAT["trap"]]
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]] > 0
    assert st[STAT["inj_reply"]] == st[STAT["ej_reply"]]


@pytest.mark.parametrize("flags", FLAG_SETS[:2], ids=["interleaved", "central"])
def test_checkpoint_resumes_exactly(flags):
    rng = random.Random(99 + flags)
    p = _params(rng, 4, 4, flags, reply_flits=2)
    a = O.OracleSim(p)
    da = a.step(1500, digests=True)
    b = O.OracleSim(p)
    b.step(777)
    c = O.OracleSim(p)
    c.load(b.dump())
    assert (c.step(723, digests=True) == da[777:]).all()
    assert (c.dump() == a.dump()).all()
    with pytest.raises(Exception):
        O.OracleSim(p.with_(flags=flags ^ CENTRAL)).load(b.dump())


def test_central_directory_is_one_tile():
    """With LSPD_CENTRAL every directory access goes to the centre tile (1,1) of a 3x3 mesh,
    whose checksum alone changes; traps and evictions still keep the one-copy rule."""
    rng = random.Random(4)
    p = _params(rng, 3, 3, LSPD | CENTRAL)
    sim = O.OracleSim(p)
    sim.step(2000, check=True)
    core = split_dump(sim.dump(), p)["core"]
    nz = [t for t in range(9) if core[t, CORE["dir_sum_lo"]] != 0 or core[t, CORE["dir_sum_hi"]] != 0]
    assert nz == [4]
    assert sim.stat("dir_access") > 0
