"""Per-cycle flit-event trace of a small chip: a debug mode.

`trace(sim, cycles)` steps a chip one cycle at a time and lists what every flit did in each
cycle, derived from the canonical link state before and after the cycle (`sim_dump`'s input
slots: the flits each router arbitrates in that cycle).  A flit is named by (source, injection
cycle), which is unique (a tile injects at most one flit per cycle).  Any simulator object
with `params`, `cycle`, `step(1)` and `dump()` can be traced, so the same events come from the
HIP library's `Sim` and from the serial oracle, and can be compared one by one.

Events, in (cycle, tile, ...) order, as tuples (cycle, kind, src, inject_cycle, dst, tile, port,
deflected):
  'inject'  the flit entered the network at router `tile` in this cycle (port = -1);
  'hop'     it left router `tile` by output port `port` (0 north, 1 south, 2 east, 3 west)
            towards the neighbour's input slot; `deflected` when the hop does not bring it
            closer to its destination (Sec. 4.2: a deflection);
  'eject'   it left the network at router `tile`, its destination (port = 4).
Only chips of at most MAX_TILES tiles with one cycle per hop (router delay 1) are traced.
"""
from __future__ import annotations

import numpy as np

MAX_TILES = 64
DIRS = ((0, -1), (0, 1), (1, 0), (-1, 0))  # output ports 0..3: north, south, east, west


def _inputs(buf: np.ndarray, n: int) -> dict:
    """{(src, inject_cycle): (tile, input port, dst)} of the flits in the dump's input slots."""
    links = buf[16:16 + n * 16].reshape(n, 4, 4)
    out = {}
    for t, p in zip(*np.nonzero(links[:, :, 0] >= 0)):
        dst, inj, src = int(links[t, p, 0]), int(links[t, p, 1]) & 0x7FFFFFFF, int(links[t, p, 2])
        out[(src, inj)] = (int(t), int(p), dst)
    return out


def trace(sim, cycles: int) -> list:
    p = sim.params
    w, h = p.width, p.height
    n = w * h
    if n > MAX_TILES:
        raise ValueError(f"flit trace is for chips of at most {MAX_TILES} tiles")
    if max(1, getattr(p, "router_delay", 1)) != 1:
        raise ValueError("flit trace needs one cycle per hop (router delay 1)")

    def dist(a, b):
        return abs(a % w - b % w) + abs(a // w - b // w)

    events = []
    before = _inputs(sim.dump(), n)
    for _ in range(cycles):
        c = int(sim.cycle)
        sim.step(1)
        after = _inputs(sim.dump(), n)
        cyc = []
        seen = set()
        for key, (t2, q2, dst) in after.items():
            # the flit sits in input slot q2 of t2: it came from the neighbour in direction q2
            dx, dy = DIRS[q2]
            t = t2 + dx + dy * w
            port = q2 ^ 1  # the sending router's output port points back the other way
            if key not in before:
                if key[1] != c:
                    raise AssertionError(f"flit {key} appeared in cycle {c} without being injected")
                cyc.append((c, "inject", key[0], key[1], dst, t, -1, False))
            elif before[key][0] != t:
                raise AssertionError(f"flit {key} jumped from tile {before[key][0]} to {t2} in cycle {c}")
            cyc.append((c, "hop", key[0], key[1], dst, t, port, dist(t2, dst) >= dist(t, dst)))
            seen.add(key)
        for key, (t, _, dst) in before.items():
            if key not in seen:
                if t != dst:
                    raise AssertionError(f"flit {key} vanished at tile {t} in cycle {c}, not its destination {dst}")
                cyc.append((c, "eject", key[0], key[1], dst, t, 4, False))
        cyc.sort(key=lambda e: (e[5], {"inject": 0, "hop": 1, "eject": 1}[e[1]], e[6], e[2], e[3]))
        events.extend(cyc)
        before = after
    return events
