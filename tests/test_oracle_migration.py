"""Pins of the oracle's block migration and redirection (Sec. 3.3) on the LSPD directory model.

A block's L2 way keeps the last accessor and how many accesses in a row came from it; when a
remote tile's run reaches mig_threshold the owner sends it the block (16 flits, Table 1) and
keeps a forwarding pointer, so a request that still reaches it is redirected (1 flit); the new
owner claims the directory entry and its op completes with the directory's acknowledgement.
Checked against hand-worked latencies, the one-copy rule and requester accounting every cycle,
the directory = slice contents after a drain, and the counting identities.
"""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import CORE, STAT, quiet_params, split_dump
from tests.test_oracle_lspd import M, _run_ops

LSPD, CENTRAL = W.LSPD, W.LSPD_CENTRAL


def test_hand_trace_migration_and_redirection():
    """2x2, line 5 (directory at tile 1), threshold 2, a one-line L1.  Tile 0 brings it from
    memory (M + 4).  Tile 3 reads it remotely (11): run (3, 1) at the owner.  Tile 3 reads line
    7 (its own directory: 1 + M), which pushes 5 out of its L1.  Tile 3 reads 5 again: the
    access at the owner makes the run (3, 2), so the block migrates: 16 flits leave tile 0 from
    the cycle of the lookup (8 cycles after issue), the last arrives 2 hops later (25), the slice
    takes it the next cycle (26) and claims the entry at tile 1 (1 hop, applied at 28), whose
    acknowledgement arrives at 29: the L1 fill completes the op at 30.  Tile 2 asks for 5 twenty
    cycles into that: the directory still names tile 0 (24), tile 0 redirects the request to
    tile 3 (29, arrives 30), which serves it (33): 15."""
    p = quiet_params(2, 2, l1_lat=1, mem_lat=M, flags=LSPD, mig_threshold=2, l1_sets=1, l1_ways=1)
    sim = O.OracleSim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    assert _run_ops(sim, [(sim.cycle + 2, 3, 5)]) == {0: 11}
    assert _run_ops(sim, [(sim.cycle + 2, 3, 7)]) == {0: 1 + M}
    c0 = sim.cycle + 2
    assert _run_ops(sim, [(c0, 3, 5), (c0 + 20, 2, 5)]) == {0: 30, 1: 15}
    st = sim.stats()
    assert st[STAT["migrations"]] == 1 and st[STAT["redirects"]] == 1 and st[STAT["trap"]] == 0
    d = split_dump(sim.dump(), p)
    assert d["loc"][5] == 3
    assert 5 in d["l2"][3].ravel() and 5 not in d["l2"][0].ravel()
    assert d["core"][0, CORE["fwd_line"]] == 5 and d["core"][0, CORE["fwd_dst"]] == 3
    way = d["l2"][3].ravel().tolist().index(5)
    rec = int(d["l2rec"][3].ravel()[way])
    assert (rec & 0xFFFFF, rec >> 20) == (2, 1)   # the last access, tile 2's, once in a row


def test_threshold_zero_is_no_migration():
    rng = random.Random(2)
    p = W.SimParams(width=4, height=4, seed=rng.randrange(1 << 30), l1_sets=4, l1_ways=2, l2_sets=4, l2_ways=2,
                    mem_lat=20, op_thr=W.thr(0.5), shared_thr=W.thr(0.7), bg_thr=W.thr(0.1), shared_lines=64,
                    private_lines=16, zipf_shared_s=0.8, zipf_private_s=0.8, flags=LSPD)
    a = O.OracleSim(p).step(1500, digests=True)
    b = O.OracleSim(p.with_(mig_threshold=0)).step(1500, digests=True)
    c = O.OracleSim(p.with_(mig_threshold=1)).step(1500, digests=True)
    assert (a == b).all() and (a != c).any()


def _params(rng, w, h, flags, thr, **kw):
    base = dict(width=w, height=h, seed=rng.randrange(1 << 40), l1_sets=2, l1_ways=1, l2_sets=4, l2_ways=2,
                l1_lat=rng.choice([1, 2]), mem_lat=rng.choice([5, 30]), op_thr=W.thr(0.5), shared_thr=W.thr(0.7),
                bg_thr=W.thr(0.1), shared_lines=32, private_lines=16, zipf_shared_s=0.8, zipf_private_s=0.8,
                flags=flags, mig_threshold=thr)
    base.update(kw)
    return W.SimParams(**base)


@pytest.mark.parametrize("flags", [LSPD, LSPD | CENTRAL, LSPD | W.HIT_UNDER_MISS | W.INJECT_DELAY | W.AGE_DEFLECT],
                         ids=["interleaved", "central", "with_variants"])
@pytest.mark.parametrize("thr", [1, 2, 4])
@pytest.mark.parametrize("w,h,flits", [(2, 2, 1), (3, 3, 4), (5, 4, 2)])
def test_invariants_drain_and_identities(flags, thr, w, h, flits):
    """Every cycle: at most one slice holds a block, and the directory names it unless that
    slice is waiting for its claim to be acknowledged; requester accounting (claims and
    migrating blocks included); conservation.  After a drain: the directory equals the slices'
    contents, requests made = received, directory accesses = slice misses + traps, and every
    remote access was answered with a block, a migration, a redirection or a trap."""
    rng = random.Random(thr * 1000 + flags + 10 * w + h)
    p = _params(rng, w, h, flags, thr, reply_flits=flits)
    sim = O.OracleSim(p)
    sim.step(2000, check=True)
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
    assert {i: int(o) for i, o in enumerate(d["loc"].tolist()) if o >= 0} == held
    assert st[STAT["req_made"]] == st[STAT["req_received"]]
    assert st[STAT["dir_access"]] == st[STAT["l2_miss"]] + st[STAT["trap"]]
    answered = st[STAT["reply_sent"]] + st[STAT["migrations"]] + st[STAT["redirects"]]
    assert st[STAT["req_received"]] <= answered + st[STAT["trap"]]
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]] > 0
    if thr == 1:
        assert st[STAT["migrations"]] > 0


@pytest.mark.parametrize("flags", [LSPD, LSPD | CENTRAL], ids=["interleaved", "central"])
def test_checkpoint_mid_migration_resumes_exactly(flags):
    rng = random.Random(7 + flags)
    p = _params(rng, 4, 4, flags, 1, reply_flits=2)
    b = O.OracleSim(p)
    for _ in range(3000):   # the first cycle with a claim waiting for its acknowledgement
        b.step(1)
        core = split_dump(b.dump(), p)["core"]
        if ((core[:, CORE["state"]] == 3) & (core[:, CORE["claim"]] >= 0)).any():
            break
    else:
        raise AssertionError("no pending claim seen")
    k = b.cycle
    snap = b.dump()
    a = O.OracleSim(p)
    da = a.step(k + 800, digests=True)
    c = O.OracleSim(p)
    c.load(snap)
    assert (c.step(800, digests=True) == da[k:]).all()
    assert (c.dump() == a.dump()).all()
    with pytest.raises(Exception):
        O.OracleSim(p.with_(mig_threshold=2)).load(snap)


def test_one_remote_user_pulls_the_block():
    """A tile that keeps missing on a line homed elsewhere (a one-way L1 and two lines that
    collide there) gets it after mig_threshold remote accesses: the block ends in its slice."""
    p = quiet_params(3, 3, l1_lat=1, mem_lat=M, flags=LSPD, mig_threshold=3, l1_sets=1, l1_ways=1)
    sim = O.OracleSim(p)
    _run_ops(sim, [(0, 0, 10)])                  # line 10 now lives in tile 0's slice
    for _ in range(3):
        _run_ops(sim, [(sim.cycle + 1, 8, 10)])  # tile 8 reads it ...
        _run_ops(sim, [(sim.cycle + 1, 8, 17)])  # ... and pushes it out of its L1 (17: its own line)
    d = split_dump(sim.dump(), p)
    assert sim.stat("migrations") == 1
    assert d["loc"][10] == 8 and 10 in d["l2"][8].ravel()


def test_migration_needs_the_directory_model():
    with pytest.raises(ValueError):
        O.OracleSim(quiet_params(2, 2, mig_threshold=2))
