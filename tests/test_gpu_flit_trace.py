"""The flit-event trace of the HIP library equals the oracle's, event by event, on both kernels."""
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import flit_trace as FT
from paper_1508_03235_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("w,h,launch", [(8, 8, (4, 4, 64, 0)), (8, 8, (8, 1, 64, 0)), (5, 7, None)])
def test_gpu_trace_equals_oracle_trace(generic, w, h, launch):
    from paper_1508_03235_amd import nocsim
    p = W.config0().with_(width=w, height=h, seed=w + 7 * h, bg_thr=W.thr(0.15), l1_sets=4, l1_ways=1, reply_flits=2)
    g = nocsim.Sim(p)
    g.set_kernel(generic)
    if launch:
        g.set_launch(*launch)
    o = O.OracleSim(p)
    g.step(30)
    o.step(30)
    assert FT.trace(g, 200) == FT.trace(o, 200)
