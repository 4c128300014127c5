"""The batch boundary on the GPU: chips joining and leaving a resident batch between steps
(simb_add / simb_remove), per-slot statistics (simb_stats), and chunks replayed as a HIP graph
(simb_set_graph).  Every chip must equal its own serial-oracle run bit for bit, whatever it
ran beside and however the chunks were launched."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W

pytestmark = pytest.mark.gpu


def chips(n, base_seed, sides):
    return [W.config1().with_(width=s, height=s, seed=base_seed + i, bg_thr=W.thr(0.02 + 0.05 * (i % 5)))
            for i, s in zip(range(n), sides)]


def oracle_dump(p, cycles):
    o = O.OracleSim(p)
    o.step(cycles)
    return o.dump(), o.stats()


def test_add_remove_between_steps():
    """A batch sized for 6 chips: chips join and leave between steps, slots are reused, and
    each chip ends equal to its oracle run of the cycles it was stepped."""
    from paper_1508_03235_amd import nocsim
    params = chips(6, 5000, [8, 16, 24, 8, 32, 16])
    sims = [nocsim.Sim(p) for p in params]
    for s in sims:
        s.set_launch(16, 16, 256, 0)
    patches = sum(nocsim.patches_of(s) for s in sims)
    b = nocsim.Batch(sims[:2], block=256, max_chips=4, max_patches=patches)
    done = [0] * 6
    b.step([120, 80])
    done[0] += 120
    done[1] += 80
    s2 = b.add(sims[2])
    s3 = b.add(sims[3])
    assert (s2, s3) == (2, 3) and b.slots == 4
    with pytest.raises(nocsim.SimError) as e:     # capacity: four chips
        b.add(sims[4])
    assert e.value.code == -5
    b.step([50, 0, 200, 33])
    done[0] += 50
    done[2] += 200
    done[3] += 33
    b.remove(0)
    assert b.add(sims[4]) == 0                     # the freed slot is reused
    b.remove(sims[1])
    assert b.add(sims[5]) == 1
    b.step({0: 90, 1: 140, 2: 10, 3: 0})
    done[4] += 90
    done[5] += 140
    done[2] += 10
    with pytest.raises(nocsim.SimError):
        b.remove(7)
    for i, (p, s) in enumerate(zip(params, sims)):
        assert s.cycle == done[i]
        d, st = oracle_dump(p, done[i])
        assert (s.dump() == d).all(), f"chip {i} ({p.width}x{p.height}) after {done[i]} cycles"
    # per-slot statistics are the chip's own
    for slot, i in ((0, 4), (1, 5), (2, 2), (3, 3)):
        assert np.array_equal(b.stats(slot), sims[i].stats())
    b.close()


@pytest.mark.parametrize("block,patch", [(256, 16), (64, 8)])
def test_graph_replay_equals_launches_and_oracle(block, patch):
    """The same chips stepped by graph replay of one chunk and by chunk-by-chunk launches end
    bit-identical, and equal to the oracle; includes chips of several patches (cooperative
    nodes) and uneven cycle counts that stop inside a chunk."""
    from paper_1508_03235_amd import nocsim
    params = chips(5, 6000, [8, 24, 16, 32, 8])
    cycles = [700, 1234, 999, 1500, 1]
    runs = []
    for graph in (False, True):
        sims = [nocsim.Sim(p) for p in params]
        for s in sims:
            s.set_launch(patch, patch, block, 500)
        b = nocsim.Batch(sims, block=block, graph=graph)
        b.step(cycles)
        b.step([300, 0, 301, 2, 499])
        runs.append([s.dump() for s in sims])
        b.close()
    for i, p in enumerate(params):
        assert (runs[0][i] == runs[1][i]).all(), f"chip {i}: graph replay differs from launches"
        total = cycles[i] + [300, 0, 301, 2, 499][i]
        d, _ = oracle_dump(p, total)
        assert (runs[1][i] == d).all(), f"chip {i} differs from the oracle"


def test_graph_rebuilt_after_membership_change():
    """A graph batch whose members change between steps keeps every chip exact."""
    from paper_1508_03235_amd import nocsim
    params = chips(4, 7000, [16, 8, 24, 16])
    sims = [nocsim.Sim(p) for p in params]
    for s in sims:
        s.set_launch(16, 16, 256, 400)
    b = nocsim.Batch(sims[:2], block=256, max_chips=4, max_patches=64, graph=True)
    b.step([800, 600])
    b.add(sims[2])
    b.step([100, 0, 900])
    b.remove(1)
    b.add(sims[3])
    b.step([50, 333, 10])
    done = [950, 600, 910, 333]
    for i, (p, s) in enumerate(zip(params, sims)):
        d, _ = oracle_dump(p, done[i])
        assert (s.dump() == d).all(), f"chip {i}"
    b.close()
