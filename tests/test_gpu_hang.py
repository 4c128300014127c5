"""The time-out path of the cross-workgroup waits, forced from the host: one patch stops
advancing (as a stuck workgroup would) and the waits give up after a small number of polls.
Every workgroup must exit normally, the step must report SIM_EHANG, and a checkpoint loaded
afterwards must continue exactly as an undisturbed run."""
import pytest

from paper_1508_03235_amd import workload as W

pytestmark = pytest.mark.gpu

EHANG = -6


@pytest.mark.parametrize("generic,patch", [(False, (64, 1, 64)), (True, (16, 16, 256))])
def test_stuck_patch_reports_hang_and_checkpoint_recovers(generic, patch):
    from paper_1508_03235_amd import nocsim
    p = W.config1().with_(bg_thr=W.thr(0.05))
    ref = nocsim.Sim(p)
    ref.set_kernel(generic)
    ref.set_launch(*patch, 500)
    ref.step(700)
    want = ref.dump()

    s = nocsim.Sim(p)
    s.set_kernel(generic)
    s.set_launch(*patch, 500)
    s.step(300)
    ckpt = s.dump()
    s.force_hang(5, 420, 4096)            # patch 5 stops at cycle 420
    with pytest.raises(nocsim.SimError) as e:
        s.step(1500)                       # three launches; all of them must end
    assert e.value.code == EHANG
    with pytest.raises(nocsim.SimError) as e:
        s.stats()
    assert e.value.code == EHANG
    s.force_hang(-1, 0, 0)
    s.load(ckpt)
    s.step(400)
    assert (s.dump() == want).all()


def test_force_hang_rejects_bad_arguments():
    from paper_1508_03235_amd import nocsim
    s = nocsim.Sim(W.config0())
    for args in ((1, 0, 10), (-2, 0, 10), (0, -1, 10), (0, 5, -1)):   # a 4x4 chip is one patch
        with pytest.raises(nocsim.SimError):
            s.force_hang(*args)
