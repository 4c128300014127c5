"""Python binding of the C-ABI library libnocsim.so (include/nocsim.h).

Argument marshalling only: every step of the simulation runs in the HIP kernels.  PyTorch
provides the device memory (one uint8 tensor per chip) and the stream.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnocsim.so")

N_STATS = 64
STAT = {
    "cycles": 0, "inj_req": 1, "inj_reply": 2, "inj_bg": 3, "ej_req": 4, "ej_reply": 5,
    "ej_bg": 6, "lat_req": 7, "lat_reply": 8, "lat_bg": 9, "lat_max": 10,
    "traversals": 11, "deflections": 12, "ops_issued": 13, "ops_done": 14, "op_lat": 15,
    "l1_hit": 16, "l1_miss": 17, "l2_hit": 18, "l2_miss": 19, "req_made": 20,
    "req_received": 21, "reply_sent": 22, "reply_received": 23, "inj_blocked": 24,
    "bg_generated": 25, "op_lat_max": 26,
    "dir_access": 27, "dir_nack": 28, "trap": 29, "dir_evict": 30, "migrations": 48, "redirects": 49,
}
ERRORS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EINVARIANT", -5: "EBUSY", -6: "EHANG",
          -7: "ELIVELOCK"}


class SimError(RuntimeError):
    def __init__(self, fn, code):
        msg = f"{fn} failed: {ERRORS.get(code, code)}"
        if code == -3:
            msg += f" (hip error {_lib().sim_last_hip_error()})"
        super().__init__(msg)
        self.code = code


class SimConfig(C.Structure):
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

    @classmethod
    def from_params(cls, p) -> "SimConfig":
        return cls(width=p.width, height=p.height, seed_lo=p.seed & 0xFFFFFFFF,
                   seed_hi=(p.seed >> 32) & 0xFFFFFFFF, l1_sets=p.l1_sets, l1_ways=p.l1_ways,
                   l2_sets=p.l2_sets, l2_ways=p.l2_ways, l1_lat=p.l1_lat, mem_lat=p.mem_lat,
                   op_thr=p.op_thr, shared_thr=p.shared_thr, bg_thr=p.bg_thr,
                   shared_lines=p.shared_lines, private_lines=p.private_lines, flags=p.flags,
                   reply_flits=p.reply_flits, router_delay=p.router_delay, mig_threshold=p.mig_threshold)


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
        sig = {
            "sim_state_bytes": (sz, [C.POINTER(SimConfig)]),
            "sim_div_constants": (i32, [i32, i32, p]),
            "sim_create": (i32, [C.POINTER(SimConfig), p, p, i32, p, sz, p, C.POINTER(p)]),
            "sim_step": (i32, [p, i64, p]),
            "sim_sync": (i32, [p]),
            "sim_cycle": (i64, [p]),
            "sim_stats": (i32, [p, p]),
            "sim_dump_words": (sz, [p]),
            "sim_dump": (i32, [p, p, sz]),
            "sim_load": (i32, [p, p, sz]),
            "sim_force_op": (i32, [p, i32, i32]),
            "sim_force_bg": (i32, [p, i32, i32]),
            "sim_set_rates": (i32, [p, u32, u32]),
            "sim_force_hang": (i32, [p, i32, i32, i32]),
            "sim_set_watchdog": (i32, [p, i32]),
            "sim_set_launch": (i32, [p, i32, i32, i32, i32]),
            "sim_get_launch": (i32, [p, p, p, p, p]),
            "sim_set_kernel": (i32, [p, i32]),
            "sim_destroy": (i32, [p]),
            "sim_strerror": (C.c_char_p, [i32]),
            "sim_last_hip_error": (i32, []),
            "simb_state_bytes": (sz, [i32, i64]),
            "simb_create": (i32, [p, i32, i32, i32, i64, p, sz, p, C.POINTER(p)]),
            "simb_add": (i32, [p, p, C.POINTER(i32)]),
            "simb_remove": (i32, [p, i32]),
            "simb_slots": (i32, [p]),
            "simb_stats": (i32, [p, i32, p]),
            "simb_set_graph": (i32, [p, i32]),
            "simb_step": (i32, [p, p]),
            "simb_destroy": (i32, [p]),
            "simb_step_noalloc": (i32, [p, i32, i32, p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _L = L
    return _L


def exported_symbols():
    """Names of the functions the library must export (checked by the CPU tests)."""
    return ["sim_state_bytes", "sim_div_constants", "sim_create", "sim_step", "sim_sync", "sim_cycle", "sim_stats",
            "sim_dump_words", "sim_dump", "sim_load", "sim_force_op", "sim_force_bg",
            "sim_set_rates", "sim_force_hang", "sim_set_watchdog", "sim_set_launch", "sim_get_launch", "sim_set_kernel", "sim_destroy", "sim_strerror",
            "sim_last_hip_error", "simb_state_bytes", "simb_create", "simb_add", "simb_remove", "simb_slots",
            "simb_stats", "simb_set_graph", "simb_step", "simb_destroy", "simb_step_noalloc"]


def _check(fn, rc):
    if rc != 0:
        raise SimError(fn, rc)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def div_constants(width: int, tiles: int) -> np.ndarray:
    """The kernels' reciprocal constants for tile / width and line / tiles (sim_div_constants)."""
    out = np.zeros(4, dtype=np.uint32)
    _check("sim_div_constants", _lib().sim_div_constants(width, tiles, out.ctypes.data_as(C.c_void_p)))
    return out


def state_bytes(params) -> int:
    cfg = SimConfig.from_params(params)
    n = _lib().sim_state_bytes(C.byref(cfg))
    if n == 0:
        raise SimError("sim_state_bytes", -1)
    return int(n)


class Sim:
    """One simulated chip resident in device memory."""

    def __init__(self, params, device="cuda", stream=None):
        import torch
        self.params = params
        self._torch = torch
        self.device = torch.device(device)
        self.stream = stream
        cfg = SimConfig.from_params(params)
        nbytes = _lib().sim_state_bytes(C.byref(cfg))
        if nbytes == 0:
            raise SimError("sim_state_bytes", -1)
        self.nbytes = int(nbytes)
        self.mem = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.mem.data_ptr()
        self._base = (base + 255) // 256 * 256
        zs, zp = params.tables()
        self._zs = np.ascontiguousarray(zs, dtype=np.uint32)
        self._zp = np.ascontiguousarray(zp, dtype=np.uint32)
        h = C.c_void_p()
        rc = _lib().sim_create(C.byref(cfg), self._zs.ctypes.data_as(C.c_void_p),
                               self._zp.ctypes.data_as(C.c_void_p), len(self._zs) - 1,
                               C.c_void_p(self._base), self.nbytes, _stream_handle(stream),
                               C.byref(h))
        _check("sim_create", rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib().sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def cycle(self) -> int:
        return int(_lib().sim_cycle(self._h))

    def step(self, n: int, digests: bool = False, sync: bool = True):
        """Advance n cycles; with digests=True return the per-cycle state digests (uint64)."""
        d = None
        if digests:
            d = self._torch.zeros(max(n, 1), dtype=self._torch.int64, device=self.device)
        _check("sim_step", _lib().sim_step(self._h, n, C.c_void_p(d.data_ptr()) if d is not None else None))
        if sync:
            self.sync()
        if d is not None:
            return d[:n].cpu().numpy().view(np.uint64)
        return None

    def sync(self):
        _check("sim_sync", _lib().sim_sync(self._h))

    def stats(self) -> np.ndarray:
        out = np.zeros(N_STATS, dtype=np.int64)
        _check("sim_stats", _lib().sim_stats(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def stat(self, name: str) -> int:
        return int(self.stats()[STAT[name]])

    def dump(self) -> np.ndarray:
        n = _lib().sim_dump_words(self._h)
        buf = np.zeros(n, dtype=np.int32)
        _check("sim_dump", _lib().sim_dump(self._h, buf.ctypes.data_as(C.c_void_p), n))
        return buf

    def load(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.int32)
        _check("sim_load", _lib().sim_load(self._h, buf.ctypes.data_as(C.c_void_p), len(buf)))

    def force_op(self, tile: int, line: int):
        _check("sim_force_op", _lib().sim_force_op(self._h, tile, line))

    def force_bg(self, tile: int, dst: int):
        _check("sim_force_bg", _lib().sim_force_bg(self._h, tile, dst))

    def set_rates(self, op_thr: int, bg_thr: int):
        _check("sim_set_rates", _lib().sim_set_rates(self._h, op_thr, bg_thr))

    def force_hang(self, patch: int, cycle: int, polls: int):
        _check("sim_force_hang", _lib().sim_force_hang(self._h, patch, cycle, polls))

    def set_watchdog(self, max_age: int):
        """Debug mode: every step checks each router's flits and that none is older than max_age
        cycles (0 = off); a violation raises SimError (ELIVELOCK / EINVARIANT)."""
        _check("sim_set_watchdog", _lib().sim_set_watchdog(self._h, max_age))

    def set_launch(self, patch_w=0, patch_h=0, block=0, chunk=0):
        _check("sim_set_launch", _lib().sim_set_launch(self._h, patch_w, patch_h, block, chunk))

    def set_kernel(self, generic_only: bool):
        _check("sim_set_kernel", _lib().sim_set_kernel(self._h, 1 if generic_only else 0))

    def get_launch(self):
        v = [C.c_int32() for _ in range(4)]
        _check("sim_get_launch", _lib().sim_get_launch(self._h, *[C.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)


def patches_of(sim) -> int:
    """Workgroups (patches) the chip's current launch mapping cuts it into."""
    pw, ph, _, _ = sim.get_launch()
    return -(-sim.params.width // pw) * -(-sim.params.height // ph)


class Batch:
    """Chips advanced together by one persistent launch per chunk of cycles.

    `sims` fill slots 0..n-1; `max_chips` / `max_patches` size the launch table for chips added
    later with add() (0 = exactly the chips given).  graph=True replays each chunk as a HIP
    graph.  A chip's slot number is what step(), stats() and remove() take."""

    def __init__(self, sims=(), block: int = 0, stream=None, max_chips: int = 0, max_patches: int = 0,
                 graph: bool = False, device=None):
        import torch
        self.sims = list(sims)
        n = len(self.sims)
        patches = sum(patches_of(s) for s in self.sims)
        self.max_chips = max_chips or n
        self.max_patches = max_patches or patches
        nbytes = int(_lib().simb_state_bytes(self.max_chips, self.max_patches))
        if nbytes == 0:
            raise SimError("simb_state_bytes", -1)
        dev = device if device is not None else (self.sims[0].device if self.sims else "cuda")
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = (self.mem.data_ptr() + 255) // 256 * 256
        arr = (C.c_void_p * max(n, 1))(*[s.handle.value for s in self.sims])
        h = C.c_void_p()
        rc = _lib().simb_create(arr, n, block, max_chips, max_patches, C.c_void_p(base), nbytes,
                                _stream_handle(stream), C.byref(h))
        _check("simb_create", rc)
        self._h = h
        self.slot_of = {id(s): i for i, s in enumerate(self.sims)}
        self.members = {i: s for i, s in enumerate(self.sims)}
        if graph:
            self.set_graph(True)

    def add(self, sim) -> int:
        slot = C.c_int32()
        _check("simb_add", _lib().simb_add(self._h, sim.handle, C.byref(slot)))
        self.members[slot.value] = sim
        self.slot_of[id(sim)] = slot.value
        return slot.value

    def remove(self, sim_or_slot):
        slot = sim_or_slot if isinstance(sim_or_slot, int) else self.slot_of[id(sim_or_slot)]
        _check("simb_remove", _lib().simb_remove(self._h, slot))
        sim = self.members.pop(slot)
        self.slot_of.pop(id(sim), None)

    @property
    def slots(self) -> int:
        return int(_lib().simb_slots(self._h))

    def set_graph(self, on: bool):
        _check("simb_set_graph", _lib().simb_set_graph(self._h, 1 if on else 0))

    def stats(self, slot: int) -> np.ndarray:
        out = np.zeros(N_STATS, dtype=np.int64)
        _check("simb_stats", _lib().simb_stats(self._h, slot, out.ctypes.data_as(C.c_void_p)))
        return out

    def step(self, cycles):
        """cycles: one count for every member, a sequence in slot order (len == slots), or a
        {slot: cycles} dict (missing slots advance 0)."""
        n = self.slots
        if isinstance(cycles, dict):
            c = np.zeros(max(n, 1), dtype=np.int64)
            for k, v in cycles.items():
                c[k] = v
        else:
            c = np.ascontiguousarray(np.broadcast_to(np.asarray(cycles, dtype=np.int64), (max(n, 1),)))
        _check("simb_step", _lib().simb_step(self._h, c.ctypes.data_as(C.c_void_p)))

    def close(self):
        if getattr(self, "_h", None):
            _lib().simb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_noalloc(sims, cycles, block: int = 0, stream=None):
    """Advances sims[i] by cycles[i] cycles in one batched step that allocates no device memory
    (the library's static launch table; see simb_step_noalloc)."""
    n = len(sims)
    arr = (C.c_void_p * max(n, 1))(*[s.handle.value for s in sims])
    c = np.ascontiguousarray(np.broadcast_to(np.asarray(cycles, dtype=np.int64), (max(n, 1),)))
    _check("simb_step_noalloc", _lib().simb_step_noalloc(arr, n, block, c.ctypes.data_as(C.c_void_p),
                                                         _stream_handle(stream)))
