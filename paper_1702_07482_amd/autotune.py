"""Tile-shape autotuner for the fused stage kernel and the batched launch.

For a shape class it times every candidate (tile height, tile width, waves
per workgroup) through the C ABI on the GPU, keeps the fastest, and caches
the choice in autotune_cache.json next to this file, keyed by kind, filter
size, filter count and shape class.  Timing uses HIP events on the current
stream around repeated calls; tuning runs are never part of a timed region.
"""
from __future__ import annotations

import json
import os

import torch

from . import tnrd

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

# (tile_h, tile_w, waves): widths 16*nb use every pixel of a row's 16-pixel
# blocks (32, 48, 64); tall narrow tiles (80, 96 x 32) write the least slab ring
# per pixel that still fits the local memory with the polynomial table.
CANDIDATES = ([(th, tw, nw) for nw in (8, 4) for th in (16, 24, 32, 48, 64)
               for tw in (32, 48, 64)]
              + [(th, 32, nw) for nw in (8, 4) for th in (80, 96)])


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def _store(cache):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def shape_class(H: int, W: int) -> str:
    """Images within a factor sqrt(2) per side share a class."""
    import math
    q = lambda n: int(round(2 * math.log2(max(n, 1))))
    return f"{q(H)}x{q(W)}"


def _time(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_forward(f, model: tnrd.DeviceModel, L: int = 1, force: bool = False, verbose=False):
    """Best (tile_h, tile_w, waves) for tnrd_forward on f [N][H][W]."""
    N, H, W = f.shape
    m = model.abi()
    key = f"fwd/k{m.ksize}/nk{m.Nk}/{shape_class(H, W)}/n{min(N, 8)}"
    cache = _load()
    if key in cache and not force:
        return tuple(cache[key]["tile"])
    u = torch.empty_like(f)
    best = None
    for th, tw, nw in CANDIDATES:
        o = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, impl=tnrd.IMPL_FUSED)
        nb = tnrd.tnrd_workspace_bytes(N, H, W, m, o, 0)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=f.device)
        if tnrd.tnrd_forward(f, N, H, W, L, m, u, None, o, ws, nb) != 0:
            continue  # tile does not fit this kernel
        ms = _time(lambda: tnrd.tnrd_forward(f, N, H, W, L, m, u, None, o, ws, nb))
        if verbose:
            print(f"  tile {th}x{tw} waves {nw}: {ms:.4f} ms", flush=True)
        if best is None or ms < best[0]:
            best = (ms, (th, tw, nw))
    cache = _load()
    cache[key] = {"tile": list(best[1]), "ms": best[0]}
    _store(cache)
    return best[1]


def tune_batched(fs, looks, models, force: bool = False, verbose=False):
    """Best (tile_h, tile_w, waves) for tnrd_forward_batched on this batch."""
    m = models[0].abi()
    sig = sorted({(f.shape[0], f.shape[1]) for f in fs})
    key = f"batched/k{m.ksize}/nk{m.Nk}/" + ",".join(shape_class(h, w) for h, w in sig) + f"/b{len(fs)}"
    cache = _load()
    if key in cache and not force:
        return tuple(cache[key]["tile"])
    best = None
    for th, tw, nw in CANDIDATES:
        if th < 6 or tw < 6:
            continue
        o = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, use_graph=0)
        try:
            outs, ws = tnrd.forward_batched(fs, looks, models, opts=o)
        except RuntimeError:
            continue
        ms = _time(lambda: tnrd.forward_batched(fs, looks, models, opts=o, outs=outs, ws=ws), reps=3)
        if verbose:
            print(f"  tile {th}x{tw} waves {nw}: {ms:.3f} ms", flush=True)
        if best is None or ms < best[0]:
            best = (ms, (th, tw, nw))
    cache = _load()
    cache[key] = {"tile": list(best[1]), "ms": best[0]}
    _store(cache)
    return best[1]
