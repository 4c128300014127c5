"""Pins of the serial oracle against facts fixed outside the oracle itself.

- Philox4x32-10: the published known-answer vectors of the Random123 distribution
  (Salmon et al., SC'11).
- Routing: closed-form zero-load latency (Manhattan distance, X then Y; paper Sec. 4.2)
  for every source/destination pair of small meshes, and hand-derived traces.
- Arbitration: brute-force check of every rule of Sec. 4.3 / Sec. 6.2.1 on enumerated
  router inputs.
- Caches: a textbook Mattson LRU stack on a 1x1 chip (every home local).
- Conservation and drain: after traffic stops, requests made = received and replies
  sent = received, the equalities of the paper's statistics table (Sec. 8, Table 3).
"""
import itertools
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import (STAT, load_golden, quiet_params, run_flit_trace, run_op_trace, split_dump, CORE,
                           check_router_rules)


def make_oracle(p):
    return O.OracleSim(p)


# ---- Philox ----------------------------------------------------------------------------
PHILOX_KAT = [  # (counter, key, output) from the Random123 known-answer file
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,out", PHILOX_KAT)
def test_philox_known_answers(ctr, key, out):
    assert O.philox(ctr, key).tolist() == out


# ---- Zipf sampler ----------------------------------------------------------------------
@pytest.mark.parametrize("n,s", [(2**20, 0.8), (2**14, 0.9), (1000, 1.2)])
def test_zipf_sampler_cdf(n, s):
    """Empirical CDF of the sampler stays within one table bucket (1/K) of the exact Zipf
    CDF, plus sampling noise; the heaviest ranks match their probabilities."""
    q = W.zipf_table(n, s)
    assert q[0] == 0 and q[-1] == n and (np.diff(q.astype(np.int64)) >= 0).all()
    rng = np.random.default_rng(123)
    u = rng.integers(0, 2**32, size=2_000_000, dtype=np.uint64).astype(np.uint32)
    r = O.zipf_ranks(q, u)
    assert r.min() >= 0 and r.max() < n
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w) / w.sum()
    for k in [0, 1, 2, 5, 10, 100, 1000, n // 10, n // 2, n - 2]:
        if k >= n:
            continue
        emp = np.mean(r <= k)
        tol = 1.0 / W.ZIPF_K + 5 * np.sqrt(cdf[k] * (1 - cdf[k]) / len(u)) + 1e-9
        assert abs(emp - cdf[k]) <= tol, (k, emp, cdf[k])


# ---- zero-load routing ---------------------------------------------------------------
@pytest.mark.parametrize("w,h", [(1, 5), (5, 1), (2, 2), (3, 3), (4, 3), (8, 8)])
def test_zero_load_latency_all_pairs(w, h):
    """A lone flit takes exactly Manhattan(src, dst) cycles, without deflection."""
    p = quiet_params(w, h)
    sim = O.OracleSim(p)
    N = w * h
    pairs = [(s, d) for s in range(N) for d in range(N) if s != d]
    if len(pairs) > 600:
        pairs = random.Random(5).sample(pairs, 600)
    for s, d in pairs:
        st0 = sim.stats()
        sim.force_bg(s, d)
        man = abs(s % w - d % w) + abs(s // w - d // w)
        sim.step(man + 1, check=True)
        st = sim.stats()
        assert st[STAT["ej_bg"]] - st0[STAT["ej_bg"]] == 1, (s, d)
        assert st[STAT["lat_bg"]] - st0[STAT["lat_bg"]] == man, (s, d)
        assert st[STAT["deflections"]] == 0
        assert st[STAT["traversals"]] - st0[STAT["traversals"]] == man


def test_route_is_x_then_y():
    """On a 4x4 mesh the lone flit 0 -> 15 visits x = 1, 2, 3 on row 0, then rows 1, 2, 3."""
    p = quiet_params(4, 4)
    sim = O.OracleSim(p)
    sim.force_bg(0, 15)
    visited = []
    for _ in range(6):
        sim.step(1)
        links = split_dump(sim.dump(), p)["links"]
        occ = np.argwhere(links[:, :, 0] >= 0)
        assert len(occ) == 1
        visited.append(int(occ[0][0]))
    assert visited == [1, 2, 3, 7, 11, 15]


# ---- hand traces ----------------------------------------------------------------------
GOLD = load_golden("hand_traces.json")


@pytest.mark.parametrize("tr", GOLD["flit_traces"], ids=lambda t: t["name"])
def test_hand_flit_trace(tr):
    run_flit_trace(make_oracle, tr)


@pytest.mark.parametrize("tr", GOLD["op_traces"], ids=lambda t: t["name"])
def test_hand_op_trace(tr):
    run_op_trace(make_oracle, tr)


# ---- arbitration rules, brute force ------------------------------------------------------
def _check_arbitration(w, h, tile, flits):
    dst = [f[0] for f in flits]
    inj = [f[1] for f in flits]
    src = [f[2] for f in flits]
    port, defl = O.arbitrate(w, h, tile, dst, inj, src)
    order = sorted(range(len(flits)), key=lambda i: (inj[i], src[i]))
    check_router_rules(w, h, tile, dst, order, port, defl)


def test_arbitration_bruteforce():
    rng = random.Random(11)
    for (w, h) in [(3, 3), (4, 3), (2, 2), (1, 3)]:
        N = w * h
        for tile in range(N):
            x, y = tile % w, tile // w
            deg = (y > 0) + (y < h - 1) + (x < w - 1) + (x > 0)
            # every arrival subset size, every destination assignment for up to 2 flits,
            # random destinations and ages beyond that
            for n in range(0, deg + 1):
                if n <= 2:
                    for dsts in itertools.product(range(N), repeat=n):
                        for ages in itertools.product(range(2), repeat=n):
                            fl = [(dsts[i], ages[i], (tile + 1 + i) % N) for i in range(n)]
                            _check_arbitration(w, h, tile, fl)
                else:
                    for _ in range(3000):
                        fl = [(rng.randrange(N), rng.randrange(3), rng.randrange(N)) for _ in range(n)]
                        keys = {(a, s) for _, a, s in fl}
                        if len(keys) < n:
                            continue
                        _check_arbitration(w, h, tile, fl)
    with pytest.raises(ValueError):
        O.arbitrate(3, 3, 0, [8, 8, 8], [0, 1, 2], [1, 2, 3])  # 3 flits, corner has 2 ports


# ---- caches vs a textbook LRU stack ------------------------------------------------------
class MattsonLRU:
    """Per-set LRU stacks (Mattson et al. 1970): a W-way LRU hits iff distance < W."""

    def __init__(self, ways):
        self.ways = ways
        self.stacks = {}

    def access(self, s, line):
        st = self.stacks.setdefault(s, [])
        hit = line in st and st.index(line) < self.ways
        if line in st:
            st.remove(line)
        st.insert(0, line)
        return hit

    def contents(self, s):
        st = self.stacks.get(s, [])[: self.ways]
        return st + [-1] * (self.ways - len(st))


@pytest.mark.parametrize("s1,w1,s2,w2", [(4, 2, 8, 4), (2, 4, 4, 8), (8, 1, 8, 2)])
def test_caches_match_mattson_on_1x1(s1, w1, s2, w2):
    p = quiet_params(1, 1, l1_sets=s1, l1_ways=w1, l2_sets=s2, l2_ways=w2, mem_lat=7, l1_lat=2)
    sim = O.OracleSim(p)
    l1, l2 = MattsonLRU(w1), MattsonLRU(w2)
    rng = random.Random(s1 * 100 + w1)
    lines = [rng.choice(range(40)) for _ in range(400)]
    exp = dict(l1_hit=0, l1_miss=0, l2_hit=0, l2_miss=0, op_lat=0)
    for line in lines:
        if l1.access(line % s1, line):
            exp["l1_hit"] += 1
        else:
            exp["l1_miss"] += 1
            if l2.access(line % s2, line):
                exp["l2_hit"] += 1
                exp["op_lat"] += p.l1_lat + 1
            else:
                exp["l2_miss"] += 1
                exp["op_lat"] += p.l1_lat + p.mem_lat
        done0 = sim.stat("ops_done")
        sim.force_op(0, line)
        for _ in range(100):
            sim.step(1, check=True)
            if sim.stat("ops_done") > done0:
                break
    st = sim.stats()
    for k, v in exp.items():
        assert st[STAT[k]] == v, k
    d = split_dump(sim.dump(), p)
    for s in range(s1):
        assert d["l1"][0, s].tolist() == l1.contents(s)
    for s in range(s2):
        assert d["l2"][0, s].tolist() == l2.contents(s)


# ---- invariants, drain, checkpoint ----------------------------------------------------
def _random_params(rng, w, h):
    return W.SimParams(width=w, height=h, seed=rng.randrange(1 << 40), l1_sets=8, l1_ways=2,
                       l2_sets=16, l2_ways=4, l1_lat=rng.choice([1, 2, 3]),
                       mem_lat=rng.choice([5, 20, 200]),
                       op_thr=rng.choice([W.thr(0.05), W.thr(0.25), W.thr(0.9)]),
                       shared_thr=W.thr(rng.random()), bg_thr=rng.choice([0, W.thr(0.1), W.thr(0.5)]),
                       shared_lines=rng.choice([64, 2**10]), private_lines=rng.choice([0, 32]),
                       zipf_shared_s=0.9, zipf_private_s=0.9)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 4), (2, 2), (3, 3), (4, 5), (8, 8)])
def test_invariants_hold_under_load(w, h):
    """Every cycle: flit conservation, no flit on a missing link, the oldest flit of each
    router never deflected, no duplicate tags, L2 slice t holds only lines homed at t, and
    every waiting requester accounted for exactly once."""
    rng = random.Random(w * 10 + h)
    for _ in range(3):
        sim = O.OracleSim(_random_params(rng, w, h))
        sim.step(1500, check=True)


@pytest.mark.parametrize("w,h", [(2, 2), (3, 3), (6, 5)])
def test_drain_delivers_everything(w, h):
    """Oldest-first routing delivers every flit: once generation stops the chip drains,
    and requests made = received, replies sent = received = requests."""
    rng = random.Random(77 + w)
    p = _random_params(rng, w, h).with_(op_thr=W.thr(0.5), bg_thr=W.thr(0.3))
    sim = O.OracleSim(p)
    sim.step(2000, check=True)
    sim.set_rates(0, 0)
    for _ in range(200):
        if sim.quiescent():
            break
        sim.step(50, check=True)
    assert sim.quiescent()
    st = sim.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]] == st[STAT["reply_sent"]] == st[STAT["reply_received"]]
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]]
    for k in ("req", "reply", "bg"):
        assert st[STAT["inj_" + k]] == st[STAT["ej_" + k]]
    assert st[STAT["bg_generated"]] == st[STAT["inj_bg"]]


def test_checkpoint_resume_is_exact():
    p = W.config0()
    a = O.OracleSim(p)
    da = a.step(3000, digests=True)
    b = O.OracleSim(p)
    b.step(1234)
    snap = b.dump()
    c = O.OracleSim(p)
    c.load(snap)
    dc = c.step(3000 - 1234, digests=True)
    assert (dc == da[1234:]).all()
    assert (c.dump() == a.dump()).all()


def test_digest_tracks_state():
    p = W.config0()
    d1 = O.OracleSim(p).step(500, digests=True)
    d2 = O.OracleSim(p).step(500, digests=True)
    d3 = O.OracleSim(p.with_(seed=2)).step(500, digests=True)
    assert (d1 == d2).all()
    assert (d1 != d3).sum() > 400


def test_reduces_to_uniform_traffic_without_cache_ops():
    """With memory ops off the chip is a plain uniform-random network: every generated
    flit is background, average latency at low load is close to the mean Manhattan
    distance of a k x k mesh, (k^2 - 1) * 2 / (3k) per dimension pair."""
    k = 8
    p = quiet_params(k, k, bg_thr=W.thr(0.005), seed=9)
    sim = O.OracleSim(p)
    sim.step(20000, check=False)
    st = sim.stats()
    assert st[STAT["inj_req"]] == 0 and st[STAT["ops_issued"]] == 0
    avg = st[STAT["lat_bg"]] / st[STAT["ej_bg"]]
    # mean |dx|+|dy| over distinct ordered tile pairs of a k x k mesh
    n = k * k
    mean_man = (2 * (k * k - 1) / (3 * k)) * n / (n - 1)
    assert abs(avg - mean_man) < 0.1 * mean_man, (avg, mean_man)
    assert st[STAT["deflections"]] < 0.02 * st[STAT["traversals"]]


# ---- multi-flit reply packets (Sec. 3.6, Table 1) -------------------------------------------

def _op_latencies(p, ops, max_cycles=2000):
    """Runs forced ops one after another on a quiet chip; returns each op's latency."""
    sim = O.OracleSim(p)
    out = []
    for tile, line in ops:
        st0 = sim.stats()
        sim.force_op(tile, line)
        for _ in range(max_cycles):
            sim.step(1, check=True)
            st = sim.stats()
            if st[STAT["ops_done"]] > st0[STAT["ops_done"]]:
                break
        else:
            raise AssertionError("op did not finish")
        out.append(int(st[STAT["op_lat"]] - st0[STAT["op_lat"]]))
    return out, sim


@pytest.mark.parametrize("flits", [1, 2, 4, 16])
def test_packet_latency_adds_one_cycle_per_extra_flit(flits):
    """At zero load the F flits of a reply leave the home on consecutive cycles over the same
    free path, so the block is complete F-1 cycles after its first flit arrives: each op that
    crosses the network takes F-1 cycles longer than with one flit (the hand trace T4 gives
    205, 5 and 7 for one flit), and an L1 hit is unchanged."""
    tr = next(t for t in load_golden("hand_traces.json")["op_traces"] if t["name"] == "T4_2x2_cache_round_trip")
    p = quiet_params(tr["width"], tr["height"], l1_sets=tr["l1_sets"], l1_ways=tr["l1_ways"], l2_sets=tr["l2_sets"],
                     l2_ways=tr["l2_ways"], l1_lat=tr["l1_lat"], mem_lat=tr["mem_lat"], reply_flits=flits)
    lat, sim = _op_latencies(p, [(o["tile"], o["line"]) for o in tr["ops"]])
    want = [o["latency"] + (flits - 1 if o["latency"] > 0 else 0) for o in tr["ops"]]
    assert lat == want
    st = sim.stats()
    assert st[STAT["inj_reply"]] == st[STAT["ej_reply"]] == flits * st[STAT["reply_sent"]]
    assert st[STAT["reply_sent"]] == st[STAT["reply_received"]] == st[STAT["req_made"]]


@pytest.mark.parametrize("flits", [2, 4, 16])
@pytest.mark.parametrize("w,h", [(2, 2), (3, 3), (4, 5)])
def test_packets_keep_invariants_and_drain(w, h, flits):
    """Under load, with replies interleaving at their homes: every cycle's invariants hold
    (a queued requester's flits in flight = flits sent - flits received; a requester whose
    reply has left its home has F - received in flight), the chip drains, and reply flits
    injected = ejected = F x packets sent = F x packets received."""
    rng = random.Random(w * 100 + h + flits)
    p = _random_params(rng, w, h).with_(op_thr=W.thr(0.5), bg_thr=W.thr(0.2), reply_flits=flits)
    sim = O.OracleSim(p)
    sim.step(1500, check=True)
    sim.set_rates(0, 0)
    for _ in range(400):
        if sim.quiescent():
            break
        sim.step(50, check=True)
    assert sim.quiescent()
    st = sim.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]] == st[STAT["reply_sent"]] == st[STAT["reply_received"]] > 0
    assert st[STAT["inj_reply"]] == st[STAT["ej_reply"]] == flits * st[STAT["reply_sent"]]
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]]


def test_packets_checkpoint_mid_packet_resumes_exactly():
    """A checkpoint taken while a reply is half sent and half received resumes exactly."""
    p = W.config0().with_(reply_flits=4, op_thr=W.thr(0.5))
    b = O.OracleSim(p)
    for _ in range(3000):  # the first cycle with a packet partly sent and one partly received
        b.step(1)
        core = split_dump(b.dump(), p)["core"]
        if (core[:, CORE["node_flits_sent"]] > 0).any() and (core[:, CORE["reply_flits_received"]] > 0).any():
            break
    else:
        raise AssertionError("no partial packet in 3000 cycles")
    k = b.cycle
    snap = b.dump()
    a = O.OracleSim(p)
    da = a.step(k + 1000, digests=True)
    c = O.OracleSim(p)
    c.load(snap)
    dc = c.step(1000, digests=True)
    assert (dc == da[k:]).all()
    assert (c.dump() == a.dump()).all()


def test_single_flit_replies_are_the_default():
    p = W.config0()
    assert (O.OracleSim(p.with_(reply_flits=1)).step(800, digests=True) ==
            O.OracleSim(p.with_(reply_flits=0)).step(800, digests=True)).all()
