"""The C-ABI library loads and exports every symbol include/nocsim.h declares; host-only
calls (sizing, validation, error strings) work without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1508_03235_amd import nocsim, workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nocsim.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_\w+|simb_\w+)\s*\(", src)))


def test_header_declares_binding_surface():
    assert sorted(nocsim.exported_symbols()) == declared_functions()


def test_library_exports_every_declared_symbol():
    assert os.path.exists(nocsim.LIB_PATH), "build the library first (__graft_entry__.build())"
    out = subprocess.check_output(["nm", "-D", "--defined-only", nocsim.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = nocsim._lib()
    for f in declared_functions():
        assert hasattr(lib, f)


def test_state_bytes_and_validation():
    p = W.config2(0.05)
    n = nocsim.state_bytes(p)
    N = 208 * 208
    assert n >= N * (128 * 4 * 4 + 512 * 8 * 4)       # L1 + L2 tags
    assert n < N * 22_000
    lib = nocsim._lib()
    bad = [p.with_(l1_sets=100), p.with_(l2_ways=3), p.with_(width=0), p.with_(mem_lat=0),
           p.with_(width=2048, height=1024), p.with_(private_lines=2**20)]
    for b in bad:
        cfg = nocsim.SimConfig.from_params(b)
        assert lib.sim_state_bytes(C.byref(cfg)) == 0, b
    assert lib.sim_strerror(-6) == b"cross-workgroup wait timed out"
    assert lib.simb_state_bytes(4, 3) == 0
    assert lib.simb_state_bytes(0, 8) == 0
    # launch table (16 B per patch) and one error word per chip, each 256-byte aligned
    assert lib.simb_state_bytes(3, 20) == 512 + 256
    assert lib.simb_state_bytes(100, 1000) == 16128 + 512


def test_null_handles_rejected():
    lib = nocsim._lib()
    assert lib.sim_step(None, 1, None) == -1
    assert lib.sim_stats(None, None) == -1
    assert lib.simb_step(None, None) == -1
    assert lib.simb_stats(None, 0, None) == -1
    assert lib.simb_remove(None, 0) == -1
    assert lib.sim_set_watchdog(None, 5) == -1
    assert lib.simb_set_graph(None, 1) == -1
    assert lib.simb_slots(None) == -1
    slot = C.c_int32()
    assert lib.simb_add(None, None, C.byref(slot)) == -1
    out = C.c_void_p()
    # a batch without chips needs an explicit workgroup size and a workspace
    assert lib.simb_create(None, 0, 0, 4, 16, C.c_void_p(256), 4096, None, C.byref(out)) == -1
    assert lib.simb_create(None, 0, 64, 4, 16, None, 4096, None, C.byref(out)) == -1
    assert lib.simb_create(None, -1, 64, 4, 16, C.c_void_p(256), 4096, None, C.byref(out)) == -1


def test_zipf_tables_validated_before_any_device_work():
    """A quantile table that decreases or runs past its region is refused (no device memory is
    touched: the placeholder buffer below is never dereferenced)."""
    lib = nocsim._lib()
    p = W.config1().with_(width=4, height=4)
    cfg = nocsim.SimConfig.from_params(p)
    zs, zp = p.tables()
    out = C.c_void_p()

    def create(a, b):
        return lib.sim_create(C.byref(cfg), a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                              W.ZIPF_K, C.c_void_p(256), 1 << 30, None, C.byref(out))
    past = zp.copy()
    past[-1] = p.private_lines + 1
    assert create(zs, past) == -1
    down = zs.copy()
    down[100] = down[101] + 1
    assert create(down, zp) == -1


def test_model_options_validation():
    """Host-side validation of the model options: reply packets, variant flags, router delay,
    the directory and migration; the location array and way records are sized in."""
    lib = nocsim._lib()
    p = W.config1().with_(width=16, height=16)

    def size(q):
        return lib.sim_state_bytes(C.byref(nocsim.SimConfig.from_params(q)))

    base = size(p)
    assert base > 0
    for bad in [p.with_(reply_flits=17), p.with_(reply_flits=-1), p.with_(flags=32), p.with_(flags=W.LSPD_CENTRAL),
                p.with_(router_delay=9), p.with_(router_delay=-1), p.with_(mig_threshold=2),
                p.with_(flags=W.LSPD, mig_threshold=17)]:
        assert size(bad) == 0, bad
    for ok in [p.with_(reply_flits=16), p.with_(flags=W.AGE_DEFLECT | W.HIT_UNDER_MISS | W.INJECT_DELAY),
               p.with_(router_delay=8), p.with_(flags=W.LSPD | W.LSPD_CENTRAL),
               p.with_(flags=W.LSPD, mig_threshold=16)]:
        assert size(ok) > 0, ok
    lines = p.shared_lines + p.tiles * p.private_lines
    assert size(p.with_(flags=W.LSPD)) >= base + 4 * lines                  # location array
    ways = p.tiles * p.l2_sets * p.l2_ways
    assert size(p.with_(flags=W.LSPD, mig_threshold=3)) >= size(p.with_(flags=W.LSPD)) + 3 * 4 * ways  # way histories
    assert size(p.with_(router_delay=3)) >= base + 2 * 4 * 16 * p.tiles    # two pipeline stages


def test_product_package_never_loads_the_oracle():
    """Only the tests, the smoke check and the benchmark's CPU-baseline leg may load oracle/."""
    import ast
    import pathlib
    pkg = pathlib.Path(__file__).resolve().parent.parent / "paper_1508_03235_amd"
    for f in pkg.rglob("*.py"):
        tree = ast.parse(f.read_text())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            else:
                continue
            assert not any(n == "oracle" or n.startswith("oracle.") for n in names), f"{f} imports {names}"
