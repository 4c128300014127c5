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


def batch_candidates(side_w: int, side_h: int, block: int = 256):
    """Patch shapes for a chip inside a batch of `block`-thread workgroups (every patch at most
    `block` tiles, so that the one-tile-per-thread kernel runs it)."""
    out = []
    def add(pw, ph):
        pw, ph = min(pw, side_w), min(ph, side_h)
        if pw * ph <= block and (pw, ph) not in out:
            out.append((pw, ph))
    if side_w * side_h <= block:
        add(side_w, side_h)
    for rows in (1, 2, 4):
        if side_w * rows <= block:
            add(side_w, rows)
    for side in (8, 16):
        add(side, side)
    add(16, 8)
    add(8, 16)
    return out


def tune_batch(params_list, block: int = 256, cycles: int = 1000, warmup: int = 200, rounds: int = 1,
               verbose: bool = False):
    """Patch shape per chip shape for a batch of the given chips, measured on the device: starting
    from the largest square-ish patch of at most `block` tiles, each shape's choice is varied in
    turn (the others fixed) and the one giving the highest tile-cycles/s of the whole batch is
    kept.  Runs on scratch chips of the same parameters; returns {(width, height): (pw, ph)}."""
    import torch
    from paper_1508_03235_amd import nocsim
    shapes = sorted({(p.width, p.height) for p in params_list})
    choice = {s: batch_candidates(*s, block)[0] for s in shapes}
    for s in shapes:  # start from 16x16 (or the whole chip) where it is a candidate
        c = batch_candidates(*s, block)
        choice[s] = (min(16, s[0]), min(16, s[1])) if (min(16, s[0]), min(16, s[1])) in c else c[0]
    sims = [nocsim.Sim(p) for p in params_list]
    tiles = sum(p.tiles for p in params_list)

    def measure():
        for sim, p in zip(sims, params_list):
            pw, ph = choice[(p.width, p.height)]
            sim.set_launch(pw, ph, block, 0)
        b = nocsim.Batch(sims, block=block)
        b.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(cycles)
        dt = time.perf_counter() - t0
        b.close()
        return tiles * cycles / dt

    best = measure()
    trials = [(dict(choice), best)]
    for _ in range(rounds):
        for s in shapes:
            keep = choice[s]
            for cand in batch_candidates(*s, block):
                if cand == keep:
                    continue
                choice[s] = cand
                try:
                    v = measure()
                except nocsim.SimError:
                    continue
                trials.append((dict(choice), v))
                if verbose:
                    print(f"  {s} -> {cand}: {v:.3e} tile-cycles/s")
                if v > best:
                    best, keep = v, cand
            choice[s] = keep
    del sims
    return dict(choice), best, len(trials)


def apply_batch_mapping(sims, mapping, block: int = 256, chunk: int = 0):
    """Sets every chip's launch mapping to the tuned patch shape of its chip shape."""
    for s in sims:
        pw, ph = mapping[(s.params.width, s.params.height)]
        s.set_launch(pw, ph, block, chunk)
