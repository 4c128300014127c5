"""Helpers shared by the tests: canonical-dump views and the hand-trace runner.

The runner drives any simulator object with the common surface (step, dump, stats,
force_op, force_bg, cycle), so the same golden traces check the oracle on the CPU and
the HIP library on the GPU.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

STAT = {
    "cycles": 0, "inj_req": 1, "inj_reply": 2, "inj_bg": 3, "ej_req": 4, "ej_reply": 5,
    "ej_bg": 6, "lat_req": 7, "lat_reply": 8, "lat_bg": 9, "lat_max": 10,
    "traversals": 11, "deflections": 12, "ops_issued": 13, "ops_done": 14, "op_lat": 15,
    "l1_hit": 16, "l1_miss": 17, "l2_hit": 18, "l2_miss": 19, "req_made": 20,
    "req_received": 21, "reply_sent": 22, "reply_received": 23, "inj_blocked": 24,
    "bg_generated": 25, "op_lat_max": 26,
    "dir_access": 27, "dir_nack": 28, "trap": 29, "dir_evict": 30, "migrations": 48, "redirects": 49,
}
CORE = {"state": 0, "wake": 1, "line": 2, "issue": 3, "l2q": 4, "l2q_line": 5, "hit_head": 6,
        "hit_tail": 7, "miss_head": 8, "miss_tail": 9, "bg_pending": 10, "node_next": 11,
        "node_ready": 12, "node_line": 13, "force_line": 14, "force_dst": 15, "reply_flits_received": 16,
        "node_flits_sent": 17, "deferred_line": 18, "deferred_issue": 19, "target": 20, "pending_ev": 21,
        "dir_sum_lo": 22, "dir_sum_hi": 23, "claim": 24, "fwd_line": 25, "fwd_dst": 26, "note": 27}
N_STATS = 64


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def split_dump(buf, params):
    N = params.width * params.height
    o = 16
    out = {"header": buf[:16]}
    out["links"] = buf[o:o + N * 16].reshape(N, 4, 4); o += N * 16
    cw = int(buf[11])   # core-record words (header word 11)
    out["core"] = buf[o:o + N * cw].reshape(N, cw); o += N * cw
    n1 = N * params.l1_sets * params.l1_ways
    out["l1"] = buf[o:o + n1].reshape(N, params.l1_sets, params.l1_ways); o += n1
    n2 = N * params.l2_sets * params.l2_ways
    out["l2"] = buf[o:o + n2].reshape(N, params.l2_sets, params.l2_ways); o += n2
    out["stats"] = buf[o:o + 2 * N_STATS].copy().view(np.int64); o += 2 * N_STATS
    out["ages"] = buf[o:o + N * 4].reshape(N, 4); o += N * 4   # deflection count of each input slot's flit
    D = max(1, int(buf[13]))   # router delay: stages 1..D-1 of the routers' pipelines follow
    out["pipe"] = buf[o:o + (D - 1) * N * 16].reshape(D - 1, N, 4, 4); o += (D - 1) * N * 16
    out["pipe_ages"] = buf[o:o + (D - 1) * N * 4].reshape(D - 1, N, 4); o += (D - 1) * N * 4
    lines = params.shared_lines + N * params.private_lines if int(buf[14]) else 0
    out["loc"] = buf[o:o + lines]; o += lines   # LSPD directory: owner of each line, -1 = not on chip
    mig = int(buf[15])   # migration: each L2 way's last `mig` accessors, most recent first
    ways = N * params.l2_sets * params.l2_ways * mig
    out["l2rec"] = buf[o:o + ways].reshape(-1, params.l2_sets, params.l2_ways * mig) if ways else buf[o:o]
    return out


def check_router_rules(w, h, tile, dst, order, port, defl):
    """The arbitration rules of one router (Sec. 4.3, Sec. 6.2.1), given the priority order of
    its flits: distinct ports on the mesh; a destined flit ejects if no flit before it did;
    otherwise its first free productive port, X before Y; otherwise the lowest-numbered free
    port, counted as a deflection; so the first flit is never deflected."""
    x, y = tile % w, tile // w
    valid = [y > 0, y < h - 1, x < w - 1, x > 0]
    used = set()
    for rank, i in enumerate(order):
        p = int(port[i])
        assert p not in used, "two flits on one port"
        assert p == 4 or valid[p], "flit sent off the mesh"
        used.add(p)
        dx, dy = dst[i] % w - x, dst[i] // w - y
        prefs = ([2] if dx > 0 else [3] if dx < 0 else []) + ([1] if dy > 0 else [0] if dy < 0 else [])
        taken_before = {int(port[j]) for j in order[:rank]}
        if dst[i] == tile and 4 not in taken_before:
            assert p == 4 and not defl[i], "destined flit with a free eject must eject"
            continue
        assert p != 4, "only the first destined flit ejects"
        free_prefs = [q for q in prefs if q not in taken_before]
        if free_prefs:
            assert p == free_prefs[0] and not defl[i], "first free productive port, X before Y"
        else:
            free = [q for q in range(4) if valid[q] and q not in taken_before]
            assert p == free[0] and defl[i], "deflection to the lowest free port"
    if order:
        assert not defl[order[0]], "the first flit is never deflected"


def quiet_params(width, height, **kw):
    """A chip with no random traffic: flits and ops come only from the test hooks."""
    from paper_1508_03235_amd.workload import SimParams
    base = dict(width=width, height=height, seed=1, op_thr=0, bg_thr=0, shared_lines=2**20,
                private_lines=0)
    base.update(kw)
    return SimParams(**base)


def run_flit_trace(make_sim, tr):
    p = quiet_params(tr["width"], tr["height"])
    sim = make_sim(p)
    slots = {}
    for s in tr["slots"]:
        slots.setdefault(s["after"], []).append(s)
    injects = {}
    for i in tr["inject"]:
        injects.setdefault(i["at"], []).append(i)
    for c in range(tr["run"]):
        for i in injects.get(c, []):
            sim.force_bg(i["src"], i["dst"])
        sim.step(1)
        for s in slots.get(c + 1, []):
            d = split_dump(sim.dump(), p)
            got = d["links"][s["tile"], s["port"]].tolist()
            assert got == s["flit"], (tr["name"], s, got)
    st = sim.stats()
    for k, v in tr["stats"].items():
        assert st[STAT[k]] == v, (tr["name"], k, int(st[STAT[k]]), v)
    d = split_dump(sim.dump(), p)
    assert (d["links"][:, :, 0] < 0).all(), "network must be empty at the end"


def run_op_trace(make_sim, tr, max_cycles=1000):
    p = quiet_params(tr["width"], tr["height"], l1_sets=tr["l1_sets"], l1_ways=tr["l1_ways"],
                     l2_sets=tr["l2_sets"], l2_ways=tr["l2_ways"], l1_lat=tr["l1_lat"],
                     mem_lat=tr["mem_lat"])
    sim = make_sim(p)
    for op in tr["ops"]:
        start = sim.cycle
        st0 = sim.stats()
        sim.force_op(op["tile"], op["line"])
        checks = {}
        for s in op.get("slots", []):
            checks.setdefault(start + s["after"], []).append(("slot", s))
        for s in op.get("core", []):
            checks.setdefault(start + s["after"], []).append(("core", s))
        for _ in range(max_cycles):
            sim.step(1)
            for kind, s in checks.get(sim.cycle, []):
                d = split_dump(sim.dump(), p)
                if kind == "slot":
                    got = d["links"][s["tile"], s["port"]].tolist()
                    assert got == s["flit"], (tr["name"], s, got)
                else:
                    for k, v in s.items():
                        if k in ("after", "tile"):
                            continue
                        assert d["core"][s["tile"], CORE[k]] == v, (tr["name"], s, k, d["core"][s["tile"]].tolist())
            st = sim.stats()
            if st[STAT["ops_done"]] > st0[STAT["ops_done"]]:
                break
        else:
            raise AssertionError(f"{tr['name']}: op {op} did not finish")
        lat = int(st[STAT["op_lat"]] - st0[STAT["op_lat"]])
        assert lat == op["latency"], (tr["name"], op, lat)
    st = sim.stats()
    for k, v in tr["stats"].items():
        assert st[STAT[k]] == v, (tr["name"], k, int(st[STAT[k]]), v)
    if "final_sets" in tr:
        d = split_dump(sim.dump(), p)
        for s, ways in tr["final_sets"].get("l1", {}).items():
            assert d["l1"][0, int(s)].tolist() == ways
        for s, ways in tr["final_sets"].get("l2", {}).items():
            assert d["l2"][0, int(s)].tolist() == ways
