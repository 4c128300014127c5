"""Pins of the oracle's model variants (the flags of SimParams), on the CPU.

AGE_DEFLECT   - priority by deflection count (Sec. 4.2, Sec. 6.2.1, Sec. 7.1 phase two);
HIT_UNDER_MISS - hits served while a miss is outstanding, no miss under a miss (Sec. 3.5);
INJECT_DELAY  - a flit enters the network the cycle after it is made, through the router's
                injection register (Sec. 6.2.1, Sec. 7.1 phase three).

Each variant is checked against something other than the oracle's own code: the arbitration
rules replayed from dumps of every cycle, a closed form for a flit's deflection count, hand
latencies, and an independent model of a 1x1 chip's core written from the rules.
"""
import itertools
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import (CORE, STAT, check_router_rules, load_golden, quiet_params, split_dump)

AGE, HUM, DELAY = W.AGE_DEFLECT, W.HIT_UNDER_MISS, W.INJECT_DELAY
KIND_REQ, KIND_REPLY = 0, 1


def _params(rng, w, h, flags, **kw):
    base = dict(width=w, height=h, seed=rng.randrange(1 << 40), l1_sets=4, l1_ways=2, l2_sets=8,
                l2_ways=2, l1_lat=rng.choice([1, 2]), mem_lat=rng.choice([5, 30]), op_thr=W.thr(0.5),
                shared_thr=W.thr(0.5), bg_thr=W.thr(0.25), shared_lines=64, private_lines=16,
                zipf_shared_s=0.8, zipf_private_s=0.8, flags=flags)
    base.update(kw)
    return W.SimParams(**base)


def _man(w, a, b):
    return abs(a % w - b % w) + abs(a // w - b // w)


# ---- replay: every router's decision of every cycle, checked from the dumps ------------------
def _neighbour(w, t, p):
    return (t - w, t + w, t + 1, t - 1)[p]


def _productive(w, t, dst):
    x, y = t % w, t // w
    dx, dy = dst % w - x, dst // w - y
    return ([2] if dx > 0 else [3] if dx < 0 else []) + ([1] if dy > 0 else [0] if dy < 0 else [])


def replay(p, cycles, check_cycle=None):
    """Steps an oracle chip one cycle at a time and checks, for every router and cycle, from the
    canonical dumps before and after: the ports its flits took follow the arbitration rules in
    the variant's priority order, each flit's deflection count grew by one exactly when it was
    deflected (AGE_DEFLECT; it stays 0 otherwise), and the count equals the closed form
    (dist(here, dst) - dist(src, dst) + hops) / 2, since a productive hop brings a flit one step
    closer and any other hop takes it one step away."""
    w, h, N = p.width, p.height, p.tiles
    aged = bool(p.flags & AGE)
    sim = O.OracleSim(p)
    prev = split_dump(sim.dump(), p)
    events = {"deflected_aged_first": 0, "req_eject": {}, "reply_gap": []}
    for _ in range(cycles):
        C = sim.cycle
        st0 = sim.stats()
        sim.step(1, check=True)
        cur = split_dump(sim.dump(), p)
        st1 = sim.stats()
        links0, ages0 = prev["links"], prev["ages"]
        links1, ages1 = cur["links"], cur["ages"]
        # every flit of the dump at cycle C: its deflection count in closed form
        for t in range(N):
            for q in range(4):
                f = links0[t, q]
                if f[0] < 0:
                    assert ages0[t, q] == 0
                    continue
                hops = C - f[1]
                expect = (_man(w, t, f[0]) - _man(w, f[2], f[0]) + hops) // 2 if aged else 0
                assert ages0[t, q] == expect, (C, t, q, f.tolist(), ages0[t, q], expect)
        defl_total = 0
        for t in range(N):
            x, y = t % w, t // w
            valid = [y > 0, y < h - 1, x < w - 1, x > 0]
            flits, fage = [], []
            for q in range(4):
                if links0[t, q, 0] >= 0:
                    flits.append(links0[t, q].tolist())
                    fage.append(int(ages0[t, q]))
            out = {}
            for q in range(4):
                if valid[q]:
                    f = links1[_neighbour(w, t, q), q ^ 1]
                    if f[0] >= 0:
                        out[(int(f[1]), int(f[2]))] = (q, f.tolist(), int(ages1[_neighbour(w, t, q), q ^ 1]))
            injected = [k for k in out if k == (C, t)]
            if injected:
                flits.append(out[injected[0]][1])
                fage.append(0)
            port, defl = [], []
            for f in flits:
                key = (f[1], f[2])
                if key in out:
                    q, _, a1 = out[key]
                    port.append(q)
                    d = q not in _productive(w, t, f[0])
                    defl.append(d)
                    assert a1 == (fage[len(port) - 1] + d if aged else 0)
                else:
                    port.append(4)
                    defl.append(False)
                    if f[3] >> 30 == KIND_REQ:
                        events["req_eject"][f[2]] = C
            assert port.count(4) <= 1
            assert len(out) == len(flits) - port.count(4), "a flit appeared from nowhere"
            if aged:
                order = sorted(range(len(flits)), key=lambda i: (-fage[i], flits[i][1], flits[i][2]))
                if flits and fage[order[0]] > 0 and any(defl):
                    events["deflected_aged_first"] += 1
            else:
                order = sorted(range(len(flits)), key=lambda i: (flits[i][1], flits[i][2]))
            check_router_rules(w, h, t, [f[0] for f in flits], order, port, defl)
            defl_total += sum(defl)
            if injected:
                f = out[injected[0]][1]
                if f[3] >> 30 == KIND_REQ and check_cycle:
                    check_cycle("req", C, t, prev)
                if f[3] >> 30 == KIND_REPLY and f[0] in events["req_eject"]:
                    events["reply_gap"].append(C - events["req_eject"].pop(f[0]))
        assert st1[STAT["deflections"]] - st0[STAT["deflections"]] == defl_total
        prev = cur
    return sim, events


def test_replay_base_model_follows_injection_time_priority():
    """The replay check itself, on the base model: injection-time order and no ages."""
    rng = random.Random(1)
    replay(_params(rng, 4, 4, 0), 300)


@pytest.mark.parametrize("w,h", [(4, 4), (3, 5), (6, 2)])
def test_age_deflect_replay(w, h):
    """Priority by deflection count: every router of every cycle follows the rules in the order
    (more deflections first, then injection cycle, then source), and each flit's count equals
    the closed form.  The run must reach routers where a deflected flit outranks older ones."""
    rng = random.Random(w * 7 + h)
    sim, ev = replay(_params(rng, w, h, AGE, bg_thr=W.thr(0.4)), 400)
    assert ev["deflected_aged_first"] > 0
    assert sim.stat("deflections") > 0


def test_age_arbitration_bruteforce():
    """The exported arbitration with deflection counts, over every router of small meshes."""
    rng = random.Random(13)
    for (w, h) in [(3, 3), (4, 3), (2, 2), (1, 3)]:
        N = w * h
        for tile in range(N):
            x, y = tile % w, tile // w
            deg = (y > 0) + (y < h - 1) + (x < w - 1) + (x > 0)
            for n in range(0, deg + 1):
                cases = (itertools.product(range(N), repeat=n) if n <= 2 else
                         (tuple(rng.randrange(N) for _ in range(n)) for _ in range(2000)))
                for dsts in cases:
                    inj = [rng.randrange(3) for _ in range(n)]
                    src = [(tile + 1 + i) % N for i in range(n)]
                    age = [rng.randrange(3) for _ in range(n)]
                    port, defl = O.arbitrate(w, h, tile, list(dsts), inj, src, age)
                    order = sorted(range(n), key=lambda i: (-age[i], inj[i], src[i]))
                    check_router_rules(w, h, tile, list(dsts), order, port, defl)


@pytest.mark.parametrize("w,h", [(1, 5), (3, 3), (4, 3)])
def test_age_deflect_zero_load_is_manhattan(w, h):
    """A lone flit is never deflected, so the variant leaves zero-load latency at Manhattan."""
    p = quiet_params(w, h, flags=AGE)
    sim = O.OracleSim(p)
    N = w * h
    for s in range(N):
        for d in range(N):
            if s == d:
                continue
            st0 = sim.stats()
            sim.force_bg(s, d)
            sim.step(_man(w, s, d) + 1, check=True)
            st = sim.stats()
            assert st[STAT["lat_bg"]] - st0[STAT["lat_bg"]] == _man(w, s, d)
    assert sim.stat("deflections") == 0


# ---- injection register ------------------------------------------------------------------------
def _t4():
    return next(t for t in load_golden("hand_traces.json")["op_traces"] if t["name"] == "T4_2x2_cache_round_trip")


def _op_latencies(p, ops, max_cycles=2000):
    sim = O.OracleSim(p)
    out = []
    for tile, line in ops:
        st0 = sim.stats()
        sim.force_op(tile, line)
        for _ in range(max_cycles):
            sim.step(1, check=True)
            if sim.stat("ops_done") > st0[STAT["ops_done"]]:
                break
        else:
            raise AssertionError("op did not finish")
        out.append(int(sim.stats()[STAT["op_lat"]] - st0[STAT["op_lat"]]))
    return out, sim


@pytest.mark.parametrize("flits", [1, 4])
def test_inject_delay_adds_two_cycles_per_remote_op(flits):
    """At zero load the request waits one cycle in its router's injection register and so does
    the reply: the hand trace's remote ops (205, 5, 7 with one-flit replies) take two cycles
    more, the L1 hit none; with F-flit replies the F-1 extra cycles add on top."""
    tr = _t4()
    p = quiet_params(tr["width"], tr["height"], l1_sets=tr["l1_sets"], l1_ways=tr["l1_ways"], l2_sets=tr["l2_sets"],
                     l2_ways=tr["l2_ways"], l1_lat=tr["l1_lat"], mem_lat=tr["mem_lat"], reply_flits=flits,
                     flags=DELAY)
    lat, _ = _op_latencies(p, [(o["tile"], o["line"]) for o in tr["ops"]])
    assert lat == [o["latency"] + (2 + flits - 1 if o["latency"] > 0 else 0) for o in tr["ops"]]


@pytest.mark.parametrize("flags", [0, DELAY])
def test_inject_delay_replay(flags):
    """Under load: with the register, a request flit injected in cycle C comes from a core that
    was already waiting to send before C, and a reply leaves its home no earlier than two cycles
    after the request was ejected there (lookup in the next cycle, injection one cycle later);
    without it, one cycle suffices and is seen."""
    rng = random.Random(5)
    p = _params(rng, 4, 4, flags, bg_thr=W.thr(0.1), mem_lat=5)
    seen_same_cycle = []

    def check(kind, C, t, before):
        st = int(before["core"][t, CORE["state"]])
        if flags & DELAY:
            assert st == 2, (C, t, st)           # SEND before cycle C
        else:
            seen_same_cycle.append(st == 1)     # L1MISS: made and injected in cycle C

    _, ev = replay(p, 500, check)
    gaps = ev["reply_gap"]
    assert gaps and min(gaps) == (2 if flags & DELAY else 1)
    if not flags & DELAY:
        assert any(seen_same_cycle)


# ---- hit under miss: an independent model of a 1x1 chip's core ---------------------------------
class LRUSets:
    """Textbook LRU lists per set, most recent first."""

    def __init__(self, sets, ways):
        self.sets, self.ways, self.lists = sets, ways, {}

    def access(self, s, line, insert):
        lst = self.lists.setdefault(s, [])
        if line in lst:
            lst.remove(line)
            lst.insert(0, line)
            return True
        if insert:
            lst.insert(0, line)
            del lst[self.ways:]
        return False

    def contents(self, s):
        lst = self.lists.get(s, [])
        return lst + [-1] * (self.ways - len(lst))


def core_model_1x1(p, cycles):
    """The core of a 1x1 chip (every line is homed at its own L2 slice, so no flit is ever
    made), written from the rules: an idle core issues when its coin falls under op_thr; an L1
    hit completes at once; a miss waits l1_lat cycles, then looks up the L2 (installing on a
    miss) and fills L1 one cycle later on a hit, mem_lat cycles later on a miss.  With hit under
    miss the core also draws while its miss is outstanding (except in the fill's cycle, when
    the L1 is busy): hits complete, the first miss is held until the fill and then looked up
    again as the core's next access, counted from its first issue."""
    hum = bool(p.flags & HUM)
    zs, _ = p.tables()
    l1, l2 = LRUSets(p.l1_sets, p.l1_ways), LRUSets(p.l2_sets, p.l2_ways)
    st = dict(ops_issued=0, ops_done=0, op_lat=0, op_lat_max=0, l1_hit=0, l1_miss=0, l2_hit=0, l2_miss=0)
    state, wake, line, issue, held = "idle", 0, 0, 0, None
    key = [p.seed & 0xFFFFFFFF, p.seed >> 32]

    def done(lat):
        st["ops_done"] += 1
        st["op_lat"] += lat
        st["op_lat_max"] = max(st["op_lat_max"], lat)

    for c in range(cycles):
        r = O.philox([c, 0, 0, 0], key)
        start, busy = state, False
        if state == "fill" and wake == c:
            l1.access(line % p.l1_sets, line, True)
            done(c - issue)
            state, busy = "idle", True
        elif state == "l1miss" and wake == c:
            hit = l2.access(line % p.l2_sets, line, True)  # one tile: set = line mod S2
            st["l2_hit" if hit else "l2_miss"] += 1
            state, wake = "fill", (c + 1 if hit else c + p.mem_lat)
        elif state == "idle":
            op = None
            if held is not None:
                op, held = held, None
            elif r[0] < p.op_thr:
                st["ops_issued"] += 1
                op = (int(O.zipf_ranks(zs, np.array([r[2]], dtype=np.uint32))[0]), c)
            if op is not None:
                busy = True
                line, issue = op
                if l1.access(line % p.l1_sets, line, False):
                    st["l1_hit"] += 1
                    done(c - issue)
                else:
                    st["l1_miss"] += 1
                    state, wake = "l1miss", c + p.l1_lat
        if hum and start != "idle" and not busy and held is None and r[0] < p.op_thr:
            st["ops_issued"] += 1
            ln = int(O.zipf_ranks(zs, np.array([r[2]], dtype=np.uint32))[0])
            if l1.access(ln % p.l1_sets, ln, False):
                st["l1_hit"] += 1
                done(0)
            else:
                held = (ln, c)
    return st, l1, l2, held


@pytest.mark.parametrize("flags", [0, HUM])
@pytest.mark.parametrize("s1,w1,s2,w2,mem", [(2, 2, 4, 2, 7), (4, 1, 2, 4, 3), (1, 4, 8, 1, 12)])
def test_core_matches_independent_model_on_1x1(flags, s1, w1, s2, w2, mem):
    p = quiet_params(1, 1, l1_sets=s1, l1_ways=w1, l2_sets=s2, l2_ways=w2, mem_lat=mem, l1_lat=2,
                     op_thr=W.thr(0.6), shared_lines=48, zipf_shared_s=0.7, seed=s1 * 31 + mem, flags=flags)
    cycles = 3000
    want, l1, l2, held = core_model_1x1(p, cycles)
    sim = O.OracleSim(p)
    sim.step(cycles, check=True)
    got = sim.stats()
    for k, v in want.items():
        assert got[STAT[k]] == v, (k, int(got[STAT[k]]), v)
    d = split_dump(sim.dump(), p)
    for s in range(s1):
        assert d["l1"][0, s].tolist() == l1.contents(s)
    for s in range(s2):
        assert d["l2"][0, s].tolist() == l2.contents(s)
    assert d["core"][0, CORE["deferred_line"]] == (held[0] if held else -1)


def test_hit_under_miss_serves_more_ops():
    """Serving hits under a miss completes more ops on the same draws."""
    rng = random.Random(3)
    p = _params(rng, 3, 3, 0, bg_thr=0)
    a, b = O.OracleSim(p), O.OracleSim(p.with_(flags=HUM))
    a.step(3000, check=True)
    b.step(3000, check=True)
    assert b.stat("ops_done") > a.stat("ops_done")
    assert b.stat("l1_hit") > a.stat("l1_hit")


# ---- every variant: invariants, drain, checkpoint --------------------------------------------
FLAG_SETS = [AGE, HUM, DELAY, AGE | HUM | DELAY]


@pytest.mark.parametrize("flags", FLAG_SETS)
@pytest.mark.parametrize("w,h,flits", [(2, 2, 1), (3, 3, 4), (4, 5, 2)])
def test_variants_keep_invariants_and_drain(flags, w, h, flits):
    """Every cycle's invariants hold (conservation, the first flit of each router never
    deflected, requester accounting, cache sets), the chip drains once traffic stops, and the
    equalities of the paper's statistics table hold."""
    rng = random.Random(flags * 100 + w * 10 + h)
    p = _params(rng, w, h, flags, reply_flits=flits)
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
    assert st[STAT["l1_hit"]] + st[STAT["l1_miss"]] == st[STAT["ops_done"]]


@pytest.mark.parametrize("flags", FLAG_SETS)
def test_variants_checkpoint_resumes_exactly(flags):
    """A dump taken mid-run (with deflection counts on the links, a held op, flits in the
    injection register's wait) resumes bit for bit, and a dump of another variant is refused."""
    rng = random.Random(flags)
    p = _params(rng, 4, 4, flags, reply_flits=2)
    a = O.OracleSim(p)
    da = a.step(1200, digests=True)
    b = O.OracleSim(p)
    b.step(700)
    snap = b.dump()
    if flags & AGE:
        assert (split_dump(snap, p)["ages"] > 0).any()
    c = O.OracleSim(p)
    c.load(snap)
    assert (c.step(500, digests=True) == da[700:]).all()
    assert (c.dump() == a.dump()).all()
    other = O.OracleSim(p.with_(flags=flags ^ AGE))
    with pytest.raises(Exception):
        other.load(snap)


def test_variants_change_the_run():
    """Each flag changes the trajectory of a loaded chip (the digests part ways)."""
    rng = random.Random(9)
    p = _params(rng, 4, 4, 0)
    base = O.OracleSim(p).step(600, digests=True)
    for f in (AGE, HUM, DELAY):
        assert (O.OracleSim(p.with_(flags=f)).step(600, digests=True) != base).any(), f


def test_unknown_flags_are_refused():
    with pytest.raises(ValueError):
        O.OracleSim(quiet_params(2, 2, flags=32))
    with pytest.raises(ValueError):
        O.OracleSim(quiet_params(2, 2, flags=W.LSPD_CENTRAL))   # central needs the directory


# ---- router delay: every hop takes D cycles ----------------------------------------------------
@pytest.mark.parametrize("D", [2, 3, 5])
@pytest.mark.parametrize("w,h", [(1, 5), (3, 3), (4, 3)])
def test_router_delay_zero_load_is_d_times_manhattan(w, h, D):
    """A lone flit spends D-1 cycles in each router's pipeline after every hop, so its
    latency is exactly D x Manhattan, without deflection."""
    p = quiet_params(w, h, router_delay=D)
    sim = O.OracleSim(p)
    N = w * h
    for s in range(N):
        for d in range(N):
            if s == d:
                continue
            st0 = sim.stats()
            sim.force_bg(s, d)
            sim.step(D * _man(w, s, d) + 1, check=True)
            st = sim.stats()
            assert st[STAT["ej_bg"]] - st0[STAT["ej_bg"]] == 1
            assert st[STAT["lat_bg"]] - st0[STAT["lat_bg"]] == D * _man(w, s, d)
    assert sim.stat("deflections") == 0


@pytest.mark.parametrize("D", [2, 4])
def test_router_delay_op_latency(D):
    """The hand trace's remote ops take 2 (D-1) cycles more per hop between requester and
    home (the request's path and the reply's), the L1 hit nothing."""
    tr = _t4()
    p = quiet_params(tr["width"], tr["height"], l1_sets=tr["l1_sets"], l1_ways=tr["l1_ways"], l2_sets=tr["l2_sets"],
                     l2_ways=tr["l2_ways"], l1_lat=tr["l1_lat"], mem_lat=tr["mem_lat"], router_delay=D)
    ops = [(o["tile"], o["line"]) for o in tr["ops"]]
    lat, _ = _op_latencies(p, ops)
    w = tr["width"]
    hops = [_man(w, t, line % (tr["width"] * tr["height"])) for t, line in ops]
    assert lat == [o["latency"] + (2 * (D - 1) * hp if o["latency"] > 0 else 0) for o, hp in zip(tr["ops"], hops)]


@pytest.mark.parametrize("flags", [0, AGE])
def test_router_delay_flits_move_on_the_beat(flags):
    """From the dumps of every cycle of a loaded chip with D = 3: a flit on a link was sent in
    a cycle congruent to its injection cycle mod D, a flit in pipeline stage k will be
    arbitrated in such a cycle, every flit counted by the statistics is in a slot or a stage,
    and (priority by deflection count) each flit's count equals the closed form with the hops
    it has made."""
    D = 3
    rng = random.Random(17 + flags)
    p = _params(rng, 4, 4, flags, router_delay=D, bg_thr=W.thr(0.35))
    w = p.width
    sim = O.OracleSim(p)
    seen_pipe = 0
    for _ in range(400):
        sim.step(1, check=True)
        C = sim.cycle
        d = split_dump(sim.dump(), p)
        st = sim.stats()
        in_flight = (st[STAT["inj_req"]] + st[STAT["inj_reply"]] + st[STAT["inj_bg"]] -
                     st[STAT["ej_req"]] - st[STAT["ej_reply"]] - st[STAT["ej_bg"]])
        count = 0
        stages = [(0, d["links"], d["ages"])] + [(k, d["pipe"][k - 1], d["pipe_ages"][k - 1]) for k in range(1, D)]
        for k, slots, ages in stages:
            for t in range(p.tiles):
                for q in range(4):
                    f = slots[t, q]
                    if f[0] < 0:
                        continue
                    count += 1
                    seen_pipe += k > 0
                    sent = C - 1 if k == 0 else C + k - 1 - D   # its last arbitration
                    assert (sent - f[1]) % D == 0, (C, k, t, q, f.tolist())
                    hops = (sent - f[1]) // D + 1
                    expect = (_man(w, t, f[0]) - _man(w, f[2], f[0]) + hops) // 2 if flags & AGE else 0
                    assert ages[t, q] == expect
        assert count == in_flight
    assert seen_pipe > 0


@pytest.mark.parametrize("D", [2, 4])
@pytest.mark.parametrize("flags", [0, AGE | HUM | DELAY])
def test_router_delay_invariants_drain_checkpoint(D, flags):
    rng = random.Random(D * 10 + flags)
    p = _params(rng, 4, 3, flags, router_delay=D, reply_flits=2)
    a = O.OracleSim(p)
    da = a.step(1200, digests=True, check=True)
    b = O.OracleSim(p)
    b.step(613)
    snap = b.dump()
    assert (split_dump(snap, p)["pipe"][..., 0] >= 0).any()
    c = O.OracleSim(p)
    c.load(snap)
    assert (c.step(587, digests=True) == da[613:]).all()
    assert (c.dump() == a.dump()).all()
    with pytest.raises(Exception):
        O.OracleSim(p.with_(router_delay=D + 1)).load(snap)
    a.set_rates(0, 0)
    for _ in range(400):
        if a.quiescent():
            break
        a.step(50, check=True)
    assert a.quiescent()
    st = a.stats()
    assert st[STAT["req_made"]] == st[STAT["req_received"]] == st[STAT["reply_sent"]] == st[STAT["reply_received"]] > 0
    assert st[STAT["ops_issued"]] == st[STAT["ops_done"]]


def test_router_delay_uniform_traffic_limit():
    """With ops off and low load the mean latency approaches D x the mean Manhattan distance."""
    k, D = 6, 2
    p = quiet_params(k, k, bg_thr=W.thr(0.004), seed=9, router_delay=D)
    sim = O.OracleSim(p)
    sim.step(20000)
    st = sim.stats()
    n = k * k
    mean_man = (2 * (k * k - 1) / (3 * k)) * n / (n - 1)
    avg = st[STAT["lat_bg"]] / st[STAT["ej_bg"]]
    assert abs(avg - D * mean_man) < 0.1 * D * mean_man, (avg, D * mean_man)


def test_router_delay_one_is_the_default():
    p = W.config0()
    assert (O.OracleSim(p.with_(router_delay=1)).step(600, digests=True) ==
            O.OracleSim(p.with_(router_delay=0)).step(600, digests=True)).all()
    with pytest.raises(ValueError):
        O.OracleSim(p.with_(router_delay=9))


def contended_pair_at_centre(age):
    """3x1 chip with priority by deflection count, at cycle 1: two background flits for the
    centre tile wait at its west and east inputs, both with the given deflection count.  In
    cycle 1 the one from tile 0 (same count and cycle, lower source) ejects and the one from
    tile 2 is deflected (Sec. 4.3, Sec. 6.2.1)."""
    p = W.config0().with_(width=3, height=1, seed=1, bg_thr=0, op_thr=0, flags=AGE)
    o = O.OracleSim(p)
    o.force_bg(0, 1)
    o.force_bg(2, 1)
    o.step(1)
    snap = o.dump()
    d = split_dump(snap, p)
    assert d["links"][1, 3, 0] == 1 and d["links"][1, 3, 2] == 0   # from tile 0, at the west input
    assert d["links"][1, 2, 0] == 1 and d["links"][1, 2, 2] == 2   # from tile 2, at the east input
    d["ages"][1, 2] = d["ages"][1, 3] = age                         # (views into the dump)
    return p, snap


def test_deflection_count_increments_and_overflow_is_reported():
    """One below the 16-bit limit the deflected flit leaves with the limit; at the limit one
    more deflection is reported as an invariant failure rather than wrapped."""
    p, snap = contended_pair_at_centre(0xFFFE)
    o = O.OracleSim(p)
    o.load(snap)
    o.step(1)
    d = split_dump(o.dump(), p)
    assert d["links"][2, 3, 2] == 2 and d["ages"][2, 3] == 0xFFFF    # back to tile 2, one more deflection
    assert o.stat("deflections") == 1 and o.stat("ej_bg") == 1
    p, snap = contended_pair_at_centre(0xFFFF)
    o = O.OracleSim(p)
    o.load(snap)
    with pytest.raises(AssertionError, match="deflection count overflow"):
        o.step(1)
