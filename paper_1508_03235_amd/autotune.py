"""Autotuner for the tile-to-thread mapping of a chip.

The step kernel's mapping is a patch shape (tiles per workgroup) and a workgroup size.  Every
mapping gives bit-identical results (randomness and tie-breaks do not depend on it), so the
tuner only measures: it runs each candidate for a short burst on a scratch chip of the same
shape, keeps the fastest, and caches the choice per (mesh shape, cache shape, device).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "nocsim", "tune.json")


def candidates(width: int, height: int, max_block: int = 256):
    """(patch_w, patch_h, block) candidates: one patch for small chips, square and strip
    patches otherwise; block = the smallest multiple of 64 covering the patch, capped."""
    n = width * height
    out = []
    def add(pw, ph):
        pw, ph = min(pw, width), min(ph, height)
        tiles = pw * ph
        for blk in sorted({min(max_block, max(64, -(-tiles // 64) * 64)), 64, 128, 256}):
            if blk <= max_block and blk <= max(64, -(-tiles // 64) * 64):
                c = (pw, ph, blk)
                if c not in out:
                    out.append(c)
    if n <= 4096:
        add(width, height)
    for side in (4, 6, 8, 10, 12, 13, 16, 20, 24, 32):
        if side < max(width, height):
            add(side, side)
    for rows in (1, 2, 4):
        add(width, rows)
    return out


def _key(params, device_name):
    return f"{device_name}|{params.width}x{params.height}|L1 {params.l1_sets}x{params.l1_ways}|L2 {params.l2_sets}x{params.l2_ways}"


def tune(params, cycles: int = 300, warmup: int = 50, cache_path: str | None = DEFAULT_CACHE,
         force: bool = False, verbose: bool = False):
    """Best (patch_w, patch_h, block) for chips shaped like `params`, measured on the device."""
    import torch
    from paper_1508_03235_amd import nocsim
    dev = torch.cuda.get_device_name(0) or "gpu"
    key = _key(params, dev)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not force:
        return tuple(cache[key]["launch"])
    results = []
    for cand in candidates(params.width, params.height):
        try:
            s = nocsim.Sim(params)
            s.set_launch(cand[0], cand[1], cand[2], max(cycles, warmup))
        except nocsim.SimError:
            continue
        s.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(cycles)
        dt = time.perf_counter() - t0
        results.append((dt, cand))
        if verbose:
            print(f"  {cand}: {params.tiles * cycles / dt:.3e} tile-cycles/s")
        del s
    if not results:
        raise RuntimeError("no launch mapping could run")
    results.sort()
    best = results[0][1]
    if cache_path:
        cache[key] = {"launch": list(best), "tile_cycles_per_s": params.tiles * cycles / results[0][0],
                      "candidates": len(results)}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best
