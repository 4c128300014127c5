"""The benchmark's roofline byte count (the scope table's algorithmic bytes per tile-cycle),
checked against a count written out link by link on small meshes."""
import numpy as np
import pytest

import bench
from paper_1508_03235_amd import workload as W
from paper_1508_03235_amd.nocsim import STAT


def directed_links(w, h):
    """Links of a w x h mesh counted one by one (each neighbour pair once in each direction)."""
    n = 0
    for y in range(h):
        for x in range(w):
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= x + dx < w and 0 <= y + dy < h:
                    n += 1
    return n


@pytest.mark.parametrize("w,h", [(1, 1), (2, 1), (2, 2), (3, 5), (208, 208)])
def test_algorithmic_bytes_per_event(w, h):
    p = W.config1().with_(width=w, height=h)
    st = np.zeros(64, dtype=np.int64)
    st[STAT["traversals"]] = 5
    st[STAT["ops_issued"]] = 3
    st[STAT["ops_done"]] = 2          # completions move no extra bytes in this count
    st[STAT["l2_hit"]] = 1
    st[STAT["l2_miss"]] = 1
    st[STAT["req_received"]] = 4
    st[STAT["reply_sent"]] = 3
    cycles = 10
    n, links = w * h, directed_links(w, h)
    # per cycle: each directed link's 4-byte destination word read and written, the core's 8-byte
    # state read and written; per event: 12 B payload written and read per traversal, 20 + 8 B per
    # L1 op, 36 + 8 B per L2 lookup, 12 B per queue append or pop
    want = cycles * (links * 8 + n * 16) + 5 * 24 + 3 * 28 + 2 * 44 + (4 + 3) * 12
    assert bench.algorithmic_bytes(p, st, cycles) == want
    assert bench.event_bytes(p, st, cycles) >= want


def test_algorithmic_bytes_of_an_oracle_run_is_near_the_scope_estimate():
    """A short oracle run of the saturated 4x4 chip (config 0): between the idle floor (links and
    core words only) and the scope table's ~150 B per tile-cycle at saturation."""
    from oracle import oracle as O
    p = W.config0()
    o = O.OracleSim(p)
    o.step(2000)
    st = o.stats()   # (the oracle's statistics block has the library's layout)
    assert all(O.STAT_NAMES[k] == STAT[k] for k in ("traversals", "ops_issued", "l2_hit", "l2_miss",
                                                     "req_received", "reply_sent"))
    per = bench.algorithmic_bytes(p, st, 2000) / (p.tiles * 2000)
    floor = (directed_links(4, 4) * 8 + 16 * 16) / 16
    assert floor < per < 160
