"""Chips above 65,536 tiles on the one-tile-per-thread kernel: with workgroups of two waves and
LDS rows sized for them (the narrow build), four workgroups share a compute unit, so a 320x320
chip's 960 row strips are all resident at once.  Parity with the serial oracle as for the
benchmark chip: per-cycle digests of a prefix (checking build) and the whole state after the
memory latency (timed build)."""
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.test_gpu_parity import assert_same_run, gpu_sim

pytestmark = pytest.mark.gpu


def big(side):
    return W.config2(0.05).with_(width=side, height=side, private_lines=2**10)  # (lines stay below 2^30)


def test_default_mapping_of_a_320x320_chip_is_row_strips():
    s = gpu_sim(big(320))
    assert s.get_launch()[:3] == (107, 1, 128)   # three strips a row, 960 workgroups


def test_320x320_prefix_digests():
    assert_same_run(big(320), 80, step_sizes=[30, 50])


def test_320x320_past_memory_latency_timed_build():
    p = big(320)
    g = gpu_sim(p)
    g.step(1200)
    o = O.OracleSim(p)
    o.step(1200)
    assert (g.dump() == o.dump()).all()


def test_benchmark_chip_keeps_its_mapping():
    assert gpu_sim(W.config2(0.05)).get_launch()[:3] == (104, 1, 128)
