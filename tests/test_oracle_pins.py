"""Pins of three oracle parts that whole-chip runs cannot tell apart from a plausible mistake.

- The home slice's L2 set index (line / N) mod S2 on chips with several homes (the reading of
  the static home, line mod N, and of its set index; the 1x1 Mattson pin cannot see it, since
  line / 1 = line there): a serialised op stream on 2x2, 4x1 and 3x1 chips against a textbook
  model of private L1s and home-slice L2s, each an LRU list per set.
- The injection order of a home's replies (a ready reply from the miss queue goes out before a
  ready reply from the hit queue): a hand trace where both become ready in one cycle at one home.
- Background destinations: drawn uniformly over the other N - 1 tiles, never the source: every
  background flit injected in a cycle is seen on a link the next cycle, and the destination
  ranks pass a chi-square test of uniformity.

Each was checked against a planted mistake in the oracle (set index line mod S2, hit replies
before miss replies, a destination draw that can name the source): each mistake fails here.
"""
import random

import numpy as np
import pytest
from scipy import stats as sps

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import STAT, load_golden, quiet_params, split_dump


# ---- L2 set index at homes of a multi-tile chip ---------------------------------------------
def textbook_caches(N, ops, s1, w1, s2, w2):
    """Private L1 per tile (set = line mod s1) and an L2 slice per home (home = line mod N,
    set = (line div N) mod s2); each set a list, most recently used first; a miss inserts at
    the front and drops the last entry (local victim selection); only L1 misses reach L2; the
    L1 is filled when the block arrives.  Ops run one at a time."""
    l1 = {}
    l2 = {}
    hits = {"l1_hit": 0, "l1_miss": 0, "l2_hit": 0, "l2_miss": 0}

    def touch(sets, key, ways, line):
        lst = sets.setdefault(key, [])
        if line in lst:
            lst.remove(line)
            lst.insert(0, line)
            return True
        lst.insert(0, line)
        del lst[ways:]
        return False

    for tile, line in ops:
        lst = l1.setdefault((tile, line % s1), [])
        if line in lst:
            hits["l1_hit"] += 1
            lst.remove(line)
            lst.insert(0, line)
            continue
        hits["l1_miss"] += 1
        home = line % N
        hits["l2_hit" if touch(l2, (home, (line // N) % s2), w2, line) else "l2_miss"] += 1
        touch(l1, (tile, line % s1), w1, line)
    return l1, l2, hits


def run_serialised(sim, ops, limit=200):
    for tile, line in ops:
        done = sim.stats()[STAT["ops_done"]]
        sim.force_op(tile, line)
        for _ in range(limit):
            sim.step(1)
            if sim.stats()[STAT["ops_done"]] > done:
                break
        else:
            raise AssertionError(f"op {tile},{line} did not finish")


@pytest.mark.parametrize("w,h", [(2, 2), (4, 1), (3, 1)])
def test_l2_set_index_is_line_over_n(w, h):
    N = w * h
    s1, w1, s2, w2 = 2, 1, 4, 2
    p = quiet_params(w, h, l1_sets=s1, l1_ways=w1, l2_sets=s2, l2_ways=w2, mem_lat=3)
    rng = random.Random(17 + N)
    pool = rng.sample(range(4096), 48)
    ops = [(rng.randrange(N), rng.choice(pool)) for _ in range(400)]
    # the pool must tell the two indexings apart on many lines
    assert sum((l // N) % s2 != l % s2 for l in pool) >= 24
    sim = O.OracleSim(p)
    run_serialised(sim, ops)
    l1, l2, hits = textbook_caches(N, ops, s1, w1, s2, w2)
    st = sim.stats()
    for k, v in hits.items():
        assert st[STAT[k]] == v, (k, int(st[STAT[k]]), v)
    d = split_dump(sim.dump(), p)
    for t in range(N):
        for s in range(s1):
            want = l1.get((t, s), [])
            assert d["l1"][t, s].tolist() == want + [-1] * (w1 - len(want)), ("L1", t, s)
        for s in range(s2):
            want = l2.get((t, s), [])
            assert d["l2"][t, s].tolist() == want + [-1] * (w2 - len(want)), ("L2", t, s)


# ---- reply injection order at a home -------------------------------------------------------
def test_ready_miss_reply_leaves_before_ready_hit_reply():
    """Hand trace (tests/golden/reply_order.json): on a 3x1 chip tile 1 is the home of lines
    = 1 mod 3.  Tile 0 misses on a cold line (lookup at a+3, reply ready a+3+M); tile 2 asks
    for a line already in the slice M cycles later (lookup and hit at a+3+M).  Both replies
    are ready in cycle a+3+M; the miss reply goes first, the hit reply one cycle later."""
    tr = load_golden("reply_order.json")
    p = quiet_params(3, 1, l1_sets=1, l1_ways=1, l2_sets=4, l2_ways=2, mem_lat=tr["mem_lat"])
    sim = O.OracleSim(p)
    lat = {}

    def op_latency_when_done(tile, before):
        st = sim.stats()
        return int(st[STAT["op_lat"]] - before[STAT["op_lat"]])

    # warm: tile 0 brings the shared line into home 1's slice
    run_serialised(sim, [(0, tr["warm_line"])])
    sim.step(5)
    a = sim.cycle
    st0 = sim.stats()
    sim.force_op(0, tr["cold_line"])
    sim.step(tr["mem_lat"])
    assert sim.cycle == a + tr["mem_lat"]
    sim.force_op(2, tr["warm_line"])
    order = []
    for _ in range(60):
        c = sim.cycle
        sim.step(1)
        d = split_dump(sim.dump(), p)
        # a reply flit leaving home 1 sits on the west (tile 0) or east (tile 2) link next cycle
        for tile, port in ((0, 2), (2, 3)):
            f = d["links"][tile, port].tolist()
            if f[0] >= 0 and f[1] == c and (f[3] >> 30) == 1:
                order.append((c - a, tile))
    st = sim.stats()
    assert st[STAT["ops_done"]] - st0[STAT["ops_done"]] == 2
    assert st[STAT["l2_hit"]] - st0[STAT["l2_hit"]] == 1 and st[STAT["l2_miss"]] - st0[STAT["l2_miss"]] == 1
    assert order == [tuple(x) for x in tr["reply_injections"]], order
    assert int(st[STAT["op_lat"]] - st0[STAT["op_lat"]]) == sum(tr["op_latencies"])
    assert int(st[STAT["op_lat_max"]]) == max(tr["op_latencies"])


# ---- background destinations ---------------------------------------------------------------
@pytest.mark.parametrize("w,h", [(4, 4), (5, 3)])
def test_background_destinations_uniform_over_other_tiles(w, h):
    N = w * h
    p = quiet_params(w, h, l1_sets=1, l1_ways=1, l2_sets=1, l2_ways=1, bg_thr=W.thr(0.25), seed=23)
    sim = O.OracleSim(p)
    ranks = np.zeros(N - 1, dtype=np.int64)
    prev = sim.stats()[STAT["inj_bg"]]
    for _ in range(2500):
        c = sim.cycle
        sim.step(1)
        d = split_dump(sim.dump(), p)
        links = d["links"].reshape(-1, 4)
        new = links[(links[:, 0] >= 0) & (links[:, 1] == c)]
        inj = sim.stats()[STAT["inj_bg"]]
        # every flit injected in cycle c left its source on a link (none addressed to itself)
        assert len(new) == inj - prev, (c, len(new), inj - prev)
        prev = inj
        src, dst = new[:, 2], new[:, 0]
        assert (src != dst).all()
        np.add.at(ranks, dst - (dst > src), 1)
    n = ranks.sum()
    assert n > 3000
    chi2 = ((ranks - n / (N - 1)) ** 2 / (n / (N - 1))).sum()
    assert chi2 < sps.chi2.ppf(1 - 1e-6, N - 2), (chi2, ranks.tolist())
