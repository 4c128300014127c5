"""Pins of the oracle's block migration and redirection (Sec. 3.3) on the LSPD directory model.

Each L2 way keeps the list of its last N accessors (N = mig_threshold); when a remote tile has
made most of them (more than half) the owner sends it the block (16 flits, Table 1) and keeps
serving the block until told of its arrival; the new owner installs it, tells the source (which
then drops its copy and keeps a forwarding pointer, so a request that still reaches it is
redirected, 1 flit) and claims the directory entry; its op completes with the directory's
acknowledgement.  Checked against hand-worked latencies, the one-copy rule (two copies only
while a block is on its way) and requester accounting every cycle, the directory = slice
contents after a drain, and the counting identities.
"""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import CORE, STAT, quiet_params, split_dump
from tests.test_oracle_lspd import M, _run_ops

LSPD, CENTRAL = W.LSPD, W.LSPD_CENTRAL


def _migrating_chip(make_sim=O.OracleSim):
    """2x2, line 5 (directory at tile 1), history of the last 2 accessors, a one-line L1.  Tile
    0 brings 5 from memory (M + 4).  Tile 3 reads it remotely (11): the owner's list of the
    block's accessors is (3, -).  Tile 3 reads line 7 (its own directory: 1 + M), which pushes
    5 out of its L1."""
    p = quiet_params(2, 2, l1_lat=1, mem_lat=M, flags=LSPD, mig_threshold=2, l1_sets=1, l1_ways=1)
    sim = make_sim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    assert _run_ops(sim, [(sim.cycle + 2, 3, 5)]) == {0: 11}
    assert _run_ops(sim, [(sim.cycle + 2, 3, 7)]) == {0: 1 + M}
    return p, sim


def test_hand_trace_migration_then_redirection(make_sim=O.OracleSim):
    """Tile 3 reads 5 again (issued at 0): L1 miss (1), own slice miss, directory access to
    tile 1 (answered at 3: tile 0 owns it), remote access reaches tile 0 at 7 and is served at
    8, where the list becomes (3, 3): both of the last two accesses are tile 3's, so the block
    migrates.  Its 16 flits leave tile 0 one per cycle from 8 (east, then south); the last
    arrives at 25; tile 3 installs the block at 26, tells tile 0 of the arrival (injected at 26)
    and claims the entry at tile 1 (injected at 27, applied at 29); the acknowledgement arrives
    at 30 and the L1 fill completes the op at 31.
    Tile 2 asks for 5 at 20: directory access at 21 (answered at 24: the entry still names tile
    0), remote access injected at 27.  At tile 2 in cycle 27 the arrival notice passing north to
    tile 0 is older, so the request is deflected east; it reaches tile 0 at 30, after the notice
    (ejected at 28, applied at 29: tile 0 dropped its copy).  Tile 0 redirects it to tile 3
    (answered at 31, at tile 2 at 32), tile 3 serves it at 35 and the fill completes at 37: 17."""
    p, sim = _migrating_chip(make_sim)
    c0 = sim.cycle + 2
    assert _run_ops(sim, [(c0, 3, 5), (c0 + 20, 2, 5)]) == {0: 31, 1: 17}
    st = sim.stats()
    assert st[STAT["migrations"]] == 1 and st[STAT["redirects"]] == 1 and st[STAT["trap"]] == 0
    d = split_dump(sim.dump(), p)
    assert d["loc"][5] == 3
    assert 5 in d["l2"][3].ravel() and 5 not in d["l2"][0].ravel()
    assert d["core"][0, CORE["fwd_line"]] == 5 and d["core"][0, CORE["fwd_dst"]] == 3   # arrival told
    assert d["core"][3, CORE["note"]] == -1
    way = d["l2"][3].ravel().tolist().index(5)
    assert d["l2rec"][3].reshape(-1, 2)[way].tolist() == [2, -1]   # tile 2's access, served at tile 3


def test_hand_trace_source_serves_during_transit(make_sim=O.OracleSim):
    """As above, but tile 2 asks at 12: directory access at 13 (answered at 16: tile 0), remote
    access injected at 19, at tile 0 at 20 and served there at 21 while the block is on its way
    to tile 3 (Sec. 3.3: the source keeps serving it until it arrives).  The reply waits in tile
    0's hit queue behind the 16 migration flits (the last injected at 23), leaves at 24 and
    reaches tile 2 at 25; the fill completes the op at 26: 14, with no redirection.  Tile 3's op
    completes at 31 as before, and tile 0 drops its copy when the arrival notice is applied."""
    p, sim = _migrating_chip(make_sim)
    c0 = sim.cycle + 2
    assert _run_ops(sim, [(c0, 3, 5), (c0 + 12, 2, 5)]) == {0: 31, 1: 14}
    st = sim.stats()
    assert st[STAT["migrations"]] == 1 and st[STAT["redirects"]] == 0 and st[STAT["trap"]] == 0
    d = split_dump(sim.dump(), p)
    assert d["loc"][5] == 3 and 5 in d["l2"][3].ravel() and 5 not in d["l2"][0].ravel()
    assert d["core"][0, CORE["fwd_line"]] == 5 and d["core"][0, CORE["fwd_dst"]] == 3


def test_hand_trace_source_evicts_the_block_on_its_way(make_sim=O.OracleSim):
    """One-way slices, history of 1.  Tile 0 owns 5 (M + 4); tile 3 reads it (issued at 0) and
    the block migrates as in the trace above (31).  Tile 0 asks for line 9 at 2: L1 miss (3),
    directory access to tile 1 (negative answer at 6), the block from memory at 26 = 2 + M + 4,
    and its install pushes 5 out of tile 0's one-way slice while 5 is still on its way (tile 3's
    arrival notice is applied at 29).  The new owner's claim updates the directory, so no
    eviction notice is sent: six requests in all (two directory accesses of tile 3 and 0 for 5
    and 9, the first op's, the remote access, the arrival notice, the claim), no directory
    eviction, and tile 0 keeps the forwarding pointer."""
    p = quiet_params(2, 2, l1_lat=1, mem_lat=M, flags=LSPD, mig_threshold=1, l1_sets=1, l1_ways=1, l2_sets=1,
                     l2_ways=1)
    sim = make_sim(p)
    assert _run_ops(sim, [(0, 0, 5)]) == {0: M + 4}
    c0 = sim.cycle + 2
    assert _run_ops(sim, [(c0, 3, 5), (c0 + 2, 0, 9)]) == {0: 31, 1: M + 4}
    st = sim.stats()
    assert st[STAT["migrations"]] == 1 and st[STAT["dir_evict"]] == 0 and st[STAT["inj_req"]] == 6
    assert st[STAT["trap"]] == 0 and st[STAT["redirects"]] == 0
    d = split_dump(sim.dump(), p)
    assert d["l2"][:, 0, 0].tolist() == [9, -1, -1, 5] and d["loc"][[5, 9]].tolist() == [3, 0]
    assert d["core"][0, CORE["fwd_line"]] == 5 and d["core"][0, CORE["fwd_dst"]] == 3


@pytest.mark.parametrize("seed", range(8))
def test_migration_races_under_pressure(seed):
    """Sec. 3.3 under heavy migration: every remote access moves its block (history of 1), few
    lines, one- or two-way slices (so that sources evict blocks that are on their way), many
    tiles asking, and with the central directory a directory tile whose own flits wait behind
    its answers (so that arrival notices are late).  Every cycle, besides the oracle's own
    checks (one copy apart from sources awaiting an arrival notice, requester accounting, no
    block received while an arrival notice is pending): no slice sends a block away while it
    waits for the directory to acknowledge its own claim of it (a block being serviced is not
    migrated).  Then the chip drains, the directory equals the slices and no slice waits for
    an arrival notice."""
    rng = random.Random(500 + seed)
    w, h = [(3, 3), (4, 4), (3, 2), (5, 3)][seed % 4]
    p = _params(rng, w, h, LSPD | (CENTRAL if seed % 2 else 0), 1, op_thr=W.thr(0.9), shared_thr=W.thr(0.95),
                shared_lines=6 + seed, private_lines=2, bg_thr=0, reply_flits=1 + seed % 3, mem_lat=5,
                l2_sets=1, l2_ways=1 + seed % 2, l1_sets=1)
    sim = O.OracleSim(p)
    saw_claim_wait = 0
    for _ in range(2000):
        sim.step(1, check=True)
        k = split_dump(sim.dump(), p)["core"]
        dst = k[:, CORE["fwd_dst"]]
        sending = (dst >= 0) & ((dst & 0x40000000) != 0)
        claiming = (k[:, CORE["state"]] == 3) & (k[:, CORE["line"]] == k[:, CORE["fwd_line"]])
        assert not (sending & claiming).any(), sim.cycle
        saw_claim_wait += int(((k[:, CORE["state"]] == 3) & (k[:, CORE["claim"]] >= 0)).sum())
    assert saw_claim_wait > 0 and sim.stat("migrations") > 50
    sim.set_rates(0, 0)
    for _ in range(200):
        if sim.quiescent():
            break
        sim.step(25, check=True)
    assert sim.quiescent()
    d = split_dump(sim.dump(), p)
    held = {int(x): t for t in range(p.tiles) for x in d["l2"][t].ravel() if x >= 0}
    assert {i: int(o) for i, o in enumerate(d["loc"].tolist()) if o >= 0} == held
    dst = d["core"][:, CORE["fwd_dst"]]
    assert not ((dst >= 0) & ((dst & 0x40000000) != 0)).any()


def remote_reads(mig, pattern, make_sim=O.OracleSim):
    """3x3, line 10 in tile 0's slice, then a read of it by each tile of `pattern` in turn; each
    reader first pushes 10 out of its one-line L1 (with a line of its own), so that the read
    reaches the slice of tile 0."""
    p = quiet_params(3, 3, l1_lat=1, mem_lat=M, flags=LSPD, mig_threshold=mig, l1_sets=1, l1_ways=1)
    sim = make_sim(p)
    _run_ops(sim, [(0, 0, 10)])
    for who in pattern:
        _run_ops(sim, [(sim.cycle + 1, who, 10 + 9 * (who + 1))])
        _run_ops(sim, [(sim.cycle + 1, who, 10)])
    return sim


def history_of_10(sim):
    d = split_dump(sim.dump(), sim.params)
    way = d["l2"][0].ravel().tolist().index(10)
    return d["l2rec"][0].reshape(-1, sim.params.mig_threshold)[way].tolist()


MAJORITY_CASES = [  # (history length, readers in order, migrations): a remote tile needs more
    (3, [8], 0),            # than half of the block's last N accesses; (8, -, -): 1 of 3
    (3, [8, 8], 1),         # (8, 8, -): 2 of 3
    (3, [8, 0, 8], 1),      # (8, 0, 8)
    (3, [8, 0, 0, 8], 0),   # (8, 0, 0): the owner's own accesses count against it
    (1, [8], 1),            # a history of 1: every remote access moves the block
    (4, [8, 8], 0),         # 2 of 4 is not more than half
    (4, [8, 4, 8, 8], 1),   # 3 of 4
]


def test_majority_of_the_last_n_accesses():
    """History of 3: a remote tile needs 2 of the block's last 3 accesses, the local core's
    accesses count against it; with a history of 1 every remote access moves the block."""
    sim = remote_reads(3, [8, 0, 4])
    assert history_of_10(sim) == [4, 0, 8] and sim.stat("migrations") == 0     # no tile made 2 of 3
    for mig, pattern, moved in MAJORITY_CASES:
        assert remote_reads(mig, pattern).stat("migrations") == moved, (mig, pattern)


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
    sim.step(2000)
    sim.set_rates(0, 0)
    for _ in range(400):
        if sim.quiescent():
            break
        sim.step(50)
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
    collide there) gets it once it has made most of the block's last accesses: with a history
    of 3, after its second remote access the block ends in its slice."""
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
