"""The flit-event trace (debug mode) on the oracle, checked against the oracle's own counters
and against the geometry of the mesh (CPU)."""
from collections import defaultdict

import pytest

from oracle import oracle as O
from paper_1508_03235_amd import flit_trace as FT
from paper_1508_03235_amd import workload as W
from tests.harness import STAT


@pytest.mark.parametrize("w,h,flags", [(5, 5, 0), (8, 8, 0), (4, 7, W.AGE_DEFLECT | W.INJECT_DELAY), (1, 6, 0), (6, 1, 0)])
def test_trace_agrees_with_counters_and_paths(w, h, flags):
    p = W.config0().with_(width=w, height=h, seed=w * 10 + h, bg_thr=W.thr(0.2), flags=flags, l1_sets=4, l1_ways=1)
    sim = O.OracleSim(p)
    sim.step(40)
    st0 = sim.stats()
    ev = FT.trace(sim, 250)
    st1 = sim.stats()
    d = {k: int(st1[STAT[k]] - st0[STAT[k]]) for k in STAT}
    kinds = defaultdict(int)
    for e in ev:
        kinds[e[1]] += 1
    assert kinds["inject"] == d["inj_req"] + d["inj_reply"] + d["inj_bg"]
    assert kinds["eject"] == d["ej_req"] + d["ej_reply"] + d["ej_bg"]
    assert kinds["hop"] == d["traversals"]
    assert sum(e[7] for e in ev) == d["deflections"]
    # a flit seen from injection to ejection: one hop per cycle from its source, ending at its
    # destination, hops = Manhattan distance + 2 x deflections (each deflection is undone)
    path = defaultdict(list)
    for e in ev:
        path[(e[2], e[3])].append(e)
    whole = 0
    for (src, inj), es in path.items():
        if es[0][1] != "inject" or es[-1][1] != "eject":
            continue
        whole += 1
        hops = [e for e in es if e[1] == "hop"]
        assert es[0][5] == src and es[-1][5] == es[-1][4]
        assert [e[0] for e in hops] == list(range(inj, inj + len(hops)))
        dst = es[-1][4]
        manhattan = abs(src % w - dst % w) + abs(src // w - dst // w)
        assert len(hops) == manhattan + 2 * sum(e[7] for e in hops)
    assert whole > 50


def test_trace_refuses_large_or_pipelined_chips():
    with pytest.raises(ValueError):
        FT.trace(O.OracleSim(W.config0().with_(width=9, height=8)), 1)
    with pytest.raises(ValueError):
        FT.trace(O.OracleSim(W.config0().with_(router_delay=2)), 1)
