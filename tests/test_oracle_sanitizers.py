"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer, and its invariant checker
firing on corrupted state (CPU only).

tests/oracle_sanitize_driver.c drives oracle/nocsim_oracle.c through every model option (the
three variants, multi-flit replies, router delays, the LSPD directory interleaved and central,
migration with histories of 1 to 3) on chips from 1x1 to 5x4, with the oracle's per-cycle
invariant checks on, a checkpoint and resume, and a drain; the build aborts on the first
sanitizer report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1508_03235_amd import workload as W
from tests.harness import split_dump

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.check_call(["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror", "-o", exe,
                           os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "nocsim_oracle.c")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok: 85 runs" in r.stdout


def _loaded(p, cycles=300):
    sim = O.OracleSim(p)
    sim.step(cycles, check=True)
    return sim


def test_checker_fires_on_a_dropped_flit():
    """Conservation: flits injected - ejected = flits on the links.  A flit removed from a slot
    of a checkpoint makes the next checked cycle fail."""
    p = W.config0().with_(width=4, height=4, seed=3, bg_thr=W.thr(0.3))
    sim = _loaded(p)
    buf = sim.dump()
    d = split_dump(buf, p)
    t, port = map(int, np.argwhere(d["links"][:, :, 0] >= 0)[0])
    off = 16 + t * 16 + port * 4
    buf[off:off + 4] = -1
    bad = O.OracleSim(p)
    bad.load(buf)
    with pytest.raises(AssertionError, match="rc=-4"):
        bad.step(1, check=True)
    good = O.OracleSim(p)
    good.load(sim.dump())
    good.step(5, check=True)


def test_checker_fires_on_a_duplicated_tag():
    """A set holds a line at most once: a checkpoint whose L2 set names one line twice fails
    the first checked cycle that uses that set (or is refused when loaded)."""
    p = W.config0().with_(width=2, height=2, seed=5, l2_sets=4, l2_ways=4, shared_lines=64)
    sim = _loaded(p, 2000)
    buf = sim.dump()
    d = split_dump(buf, p)
    n = p.tiles
    cw = int(buf[11])
    l2_off = 16 + n * 16 + n * cw + n * p.l1_sets * p.l1_ways
    sets = d["l2"]
    t, s_ = next((t, s_) for t in range(n) for s_ in range(p.l2_sets) if sets[t, s_, 0] >= 0 and sets[t, s_, 1] >= 0)
    buf[l2_off + (t * p.l2_sets + s_) * p.l2_ways + 1] = sets[t, s_, 0]
    bad = O.OracleSim(p)
    try:
        bad.load(buf)
    except Exception:
        return
    with pytest.raises(AssertionError, match="duplicate tag"):
        bad.step(3000, check=True)
