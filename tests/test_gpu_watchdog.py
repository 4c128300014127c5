"""The watchdog (debug mode, sim_set_watchdog): with a generous bound the results are those
of the plain run, on both kernels and with several patches; with a bound below the flits'
ages it stops the chip with SIM_ELIVELOCK, every workgroup exiting normally, and a checkpoint
loaded afterwards continues exactly."""
import numpy as np
import pytest

from paper_1508_03235_amd import workload as W

pytestmark = pytest.mark.gpu

ELIVELOCK = -7
CASES = [(False, (16, 1, 64)), (False, (8, 8, 64)), (True, (8, 8, 64)), (False, (32, 32, 256))]


def _chip(generic, patch, **kw):
    from paper_1508_03235_amd import nocsim
    p = W.config1().with_(width=32, height=32, bg_thr=W.thr(0.1), **kw)
    s = nocsim.Sim(p)
    s.set_kernel(generic)
    s.set_launch(*patch, 400)
    return s


@pytest.mark.parametrize("generic,patch", CASES)
def test_generous_watchdog_changes_nothing(generic, patch):
    a = _chip(generic, patch)
    da = a.step(1200, digests=True)
    b = _chip(generic, patch)
    b.set_watchdog(1 << 20)
    db = b.step(1200, digests=True)
    assert (da == db).all()
    c = _chip(generic, patch)
    c.set_watchdog(1 << 20)
    c.step(1200)                       # the checking build without a digest buffer
    assert (c.dump() == a.dump()).all() and (b.dump() == a.dump()).all()


@pytest.mark.parametrize("generic,patch", CASES)
def test_tight_watchdog_stops_the_chip(generic, patch):
    from paper_1508_03235_amd import nocsim
    s = _chip(generic, patch)
    s.step(200)
    ckpt = s.dump()
    ref = _chip(generic, patch)
    ref.step(500)
    s.set_watchdog(6)                  # flits here travel tens of cycles
    with pytest.raises(nocsim.SimError) as e:
        s.step(800)                    # two launches; both must end
    assert e.value.code == ELIVELOCK
    s.set_watchdog(0)
    s.load(ckpt)
    s.step(300)
    assert (s.dump() == ref.dump()).all()


def test_watchdog_arguments():
    from paper_1508_03235_amd import nocsim
    s = _chip(False, (16, 1, 64))
    with pytest.raises(nocsim.SimError):
        s.set_watchdog(-1)
    assert nocsim._lib().sim_strerror(ELIVELOCK).startswith(b"a flit outlived")
