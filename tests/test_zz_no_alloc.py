"""simb_step_noalloc (the batched step whose launch table lives in the library's static device
array) against the batched step with a caller workspace (simb_create + simb_step): the same chips
stepped by both end bit-identical, over two calls in a row, the second on fewer and smaller chips."""
import numpy as np
import pytest

from paper_1508_03235_amd import workload as W

pytestmark = pytest.mark.gpu


def chips(sides, base_seed, flags=0, mig=0):
    return [W.config1().with_(width=s, height=s, seed=base_seed + i, bg_thr=W.thr(0.03 + 0.04 * (i % 4)), flags=flags,
                              mig_threshold=mig, l2_sets=16 if flags else 512)
            for i, s in enumerate(sides)]


def make(params, patch):
    from paper_1508_03235_amd import nocsim
    sims = [nocsim.Sim(p) for p in params]
    for s in sims:
        s.set_launch(patch, patch, 256, 400)
    return sims


@pytest.mark.parametrize("patch", [64, 16])
@pytest.mark.parametrize("flags,mig", [(0, 0), (W.LSPD, 0), (W.LSPD, 2)], ids=["base", "directory", "migration"])
def test_noalloc_equals_workspace_batch(patch, flags, mig):
    from paper_1508_03235_amd import nocsim
    first = chips([8, 24, 16, 32, 8, 48], 9100, flags, mig)
    second_idx = [1, 4]            # the second call: fewer chips, one of them small
    c1 = [700, 1234, 999, 1500, 1, 333]
    c2 = [0, 257, 0, 0, 911, 0]
    ref = make(first, patch)
    new = make(first, patch)
    b = nocsim.Batch(ref, block=256)
    b.step(c1)
    nocsim.step_noalloc(new, c1, block=256)
    for i in range(len(first)):
        assert ref[i].cycle == new[i].cycle == c1[i]
        assert (ref[i].dump() == new[i].dump()).all(), f"first call, chip {i}"
        assert np.array_equal(ref[i].stats(), new[i].stats())
    b.step(c2)
    b.close()
    nocsim.step_noalloc([new[i] for i in second_idx], [c2[i] for i in second_idx], block=256)
    for i in range(len(first)):
        assert ref[i].cycle == new[i].cycle == c1[i] + c2[i]
        assert (ref[i].dump() == new[i].dump()).all(), f"second call, chip {i}"
        assert np.array_equal(ref[i].stats(), new[i].stats())


def test_noalloc_refuses_more_than_its_limit():
    """More chips than the static table holds: refused on the host before anything runs."""
    from paper_1508_03235_amd import nocsim
    p = W.config0()
    s = nocsim.Sim(p)
    with pytest.raises(nocsim.SimError) as e:
        nocsim.step_noalloc([s] * 1025, [1] * 1025)
    assert e.value.code == -2
    assert s.cycle == 0
    nocsim.step_noalloc([s], [10])
    assert s.cycle == 10
