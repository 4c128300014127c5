"""ctypes wrapper of the serial oracle (oracle/nocsim_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nocsim_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

N_STATS = 64
STAT_NAMES = {
    "cycles": 0, "inj_req": 1, "inj_reply": 2, "inj_bg": 3, "ej_req": 4, "ej_reply": 5,
    "ej_bg": 6, "lat_req": 7, "lat_reply": 8, "lat_bg": 9, "lat_max": 10,
    "traversals": 11, "deflections": 12, "ops_issued": 13, "ops_done": 14, "op_lat": 15,
    "l1_hit": 16, "l1_miss": 17, "l2_hit": 18, "l2_miss": 19, "req_made": 20,
    "req_received": 21, "reply_sent": 22, "reply_received": 23, "inj_blocked": 24,
    "bg_generated": 25, "op_lat_max": 26,
    "dir_access": 27, "dir_nack": 28, "trap": 29, "dir_evict": 30, "migrations": 48, "redirects": 49,
}
HIST = 32


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11, -O3)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "nocsim_oracle.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O3", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class OracleConfig(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32),
        ("seed_lo", C.c_uint32), ("seed_hi", C.c_uint32),
        ("l1_sets", C.c_int32), ("l1_ways", C.c_int32),
        ("l2_sets", C.c_int32), ("l2_ways", C.c_int32),
        ("l1_lat", C.c_int32), ("mem_lat", C.c_int32),
        ("op_thr", C.c_uint32), ("shared_thr", C.c_uint32), ("bg_thr", C.c_uint32),
        ("shared_lines", C.c_int32), ("private_lines", C.c_int32), ("flags", C.c_int32),
        ("reply_flits", C.c_int32), ("router_delay", C.c_int32), ("mig_threshold", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        p, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
        L.oracle_create.argtypes = [C.POINTER(OracleConfig), p, p, i32, C.POINTER(p)]
        L.oracle_step.argtypes = [p, i64, p, i32]
        L.oracle_stats.argtypes = [p, p]
        L.oracle_cycle.argtypes = [p]
        L.oracle_cycle.restype = i64
        L.oracle_dump_words.argtypes = [p]
        L.oracle_dump_words.restype = sz
        L.oracle_dump.argtypes = [p, p, sz]
        L.oracle_load.argtypes = [p, p, sz]
        L.oracle_force_op.argtypes = [p, i32, i32]
        L.oracle_force_bg.argtypes = [p, i32, i32]
        L.oracle_set_rates.argtypes = [p, u32, u32]
        L.oracle_quiescent.argtypes = [p]
        L.oracle_invariant_msg.argtypes = [p]
        L.oracle_invariant_msg.restype = C.c_char_p
        L.oracle_destroy.argtypes = [p]
        L.oracle_destroy.restype = None
        L.oracle_philox4x32_10.argtypes = [p, p, p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_zipf_ranks.argtypes = [p, p, i64, p]
        L.oracle_zipf_ranks.restype = None
        L.oracle_arbitrate.argtypes = [i32, i32, i32, i32, p, p, p, p, p, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def zipf_ranks(table: np.ndarray, u: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(table, dtype=np.uint32)
    uu = np.ascontiguousarray(u, dtype=np.uint32)
    out = np.zeros(len(uu), dtype=np.int32)
    lib().oracle_zipf_ranks(_ptr(t), _ptr(uu), len(uu), _ptr(out))
    return out


def arbitrate(width, height, tile, dst, inj, src, age=None):
    """(ports, deflected) for one router (age: deflection counts for the AGE_DEFLECT priority,
    None for injection-time priority); raises ValueError when there are too few ports."""
    n = len(dst)
    d = np.asarray(dst, dtype=np.int32)
    i = np.asarray(inj, dtype=np.int32)
    s = np.asarray(src, dtype=np.int32)
    a = np.asarray(age, dtype=np.int32) if age is not None else None
    port = np.zeros(max(n, 1), dtype=np.int32)
    defl = np.zeros(max(n, 1), dtype=np.int32)
    rc = lib().oracle_arbitrate(width, height, tile, n, _ptr(d), _ptr(i), _ptr(s),
                                _ptr(a) if a is not None else None, _ptr(port), _ptr(defl))
    if rc != 0:
        raise ValueError(f"arbitrate rc={rc}")
    return port[:n].copy(), defl[:n].copy()


class OracleSim:
    """One simulated chip run by the serial oracle."""

    def __init__(self, params):
        self.params = params
        zs, zp = params.tables()
        self._zs = np.ascontiguousarray(zs, dtype=np.uint32)
        self._zp = np.ascontiguousarray(zp, dtype=np.uint32)
        cfg = OracleConfig(
            width=params.width, height=params.height,
            seed_lo=params.seed & 0xFFFFFFFF, seed_hi=(params.seed >> 32) & 0xFFFFFFFF,
            l1_sets=params.l1_sets, l1_ways=params.l1_ways,
            l2_sets=params.l2_sets, l2_ways=params.l2_ways,
            l1_lat=params.l1_lat, mem_lat=params.mem_lat,
            op_thr=params.op_thr, shared_thr=params.shared_thr, bg_thr=params.bg_thr,
            shared_lines=params.shared_lines, private_lines=params.private_lines, flags=params.flags,
            reply_flits=params.reply_flits, router_delay=params.router_delay,
            mig_threshold=params.mig_threshold)
        h = C.c_void_p()
        rc = lib().oracle_create(C.byref(cfg), _ptr(self._zs), _ptr(self._zp), len(self._zs) - 1, C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_create rc={rc}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def cycle(self) -> int:
        return lib().oracle_cycle(self._h)

    def step(self, n: int, digests: bool = False, check: bool = False):
        d = np.zeros(max(n, 1), dtype=np.uint64) if digests else None
        rc = lib().oracle_step(self._h, n, _ptr(d) if d is not None else None, 1 if check else 0)
        if rc != 0:
            msg = lib().oracle_invariant_msg(self._h).decode()
            raise AssertionError(f"oracle_step rc={rc}: {msg}")
        return d[:n] if d is not None else None

    def stats(self) -> np.ndarray:
        out = np.zeros(N_STATS, dtype=np.int64)
        lib().oracle_stats(self._h, _ptr(out))
        return out

    def stat(self, name: str) -> int:
        return int(self.stats()[STAT_NAMES[name]])

    def dump(self) -> np.ndarray:
        n = lib().oracle_dump_words(self._h)
        buf = np.zeros(n, dtype=np.int32)
        rc = lib().oracle_dump(self._h, _ptr(buf), n)
        assert rc == 0
        return buf

    def load(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.int32)
        rc = lib().oracle_load(self._h, _ptr(buf), len(buf))
        if rc != 0:
            raise ValueError(f"oracle_load rc={rc}")

    def force_op(self, tile: int, line: int):
        if lib().oracle_force_op(self._h, tile, line) != 0:
            raise ValueError("force_op")

    def force_bg(self, tile: int, dst: int):
        if lib().oracle_force_bg(self._h, tile, dst) != 0:
            raise ValueError("force_bg")

    def set_rates(self, op_thr: int, bg_thr: int):
        lib().oracle_set_rates(self._h, op_thr, bg_thr)

    def quiescent(self) -> bool:
        return bool(lib().oracle_quiescent(self._h))
