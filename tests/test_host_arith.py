"""The reciprocal constants the kernels divide by (sim_div_constants), checked on the host over
their whole input range: tile / width for every width and every tile index, and line / tiles
for every chip size by the exactness condition of multiply-and-shift division (plus every line
for the benchmark chip and the largest chip)."""
import numpy as np
import pytest

from paper_1508_03235_amd import nocsim

MAX_TILES = 1 << 20      # tile indices take 20 bits
MAX_LINE = 1 << 30       # lines take 30 bits


def test_tile_over_width_every_width_every_tile():
    t = np.arange(MAX_TILES, dtype=np.uint64)
    for w in range(1, 2049):
        m = int(nocsim.div_constants(w, 1)[0])
        if w == 1:
            assert m == 0          # the kernels take tile itself as the row when width is 1
            continue
        got = (t * np.uint64(m)) >> np.uint64(32)
        assert np.array_equal(got, t // np.uint64(w)), f"width {w}"


def test_line_over_tiles_condition_every_chip_size():
    """umulhi(v, m) >> k = floor(v * m / 2^(32+k)), which equals floor(v / N) whenever
    e * v < 2^(32+k) with e = m * N - 2^(32+k) >= 0 (write v = qN + r: the fraction is
    r/N + e v / (N 2^(32+k)) < 1).  Checked for every N in [2, 2^20) at the largest line."""
    bad = []
    for n in range(2, MAX_TILES):
        c = nocsim.div_constants(1, n)
        m, k = int(c[2]), int(c[3])
        assert 0 < m < 1 << 32 and c[1] == 0
        e = m * n - (1 << (32 + k))
        if not (0 <= e and e * (MAX_LINE - 1) < 1 << (32 + k)):
            bad.append(n)
    assert not bad, bad[:10]
    assert list(nocsim.div_constants(1, 1)[2:]) == [0, 0]


@pytest.mark.parametrize("n", [43264, MAX_TILES - 1])
def test_line_over_tiles_every_line(n):
    c = nocsim.div_constants(1, n)
    m, k = np.uint64(int(c[2])), np.uint64(int(c[3]))
    chunk = 1 << 25
    for lo in range(0, MAX_LINE, chunk):
        v = np.arange(lo, lo + chunk, dtype=np.uint64)
        q = ((v * m) >> np.uint64(32)) >> k
        assert np.array_equal(q, v // np.uint64(n)), f"lines from {lo}"


def test_div_constants_rejects_bad_sizes():
    with pytest.raises(nocsim.SimError):
        nocsim.div_constants(0, 5)
    with pytest.raises(nocsim.SimError):
        nocsim.div_constants(3, 0)
