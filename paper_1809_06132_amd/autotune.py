"""Autotuner of the sweep launch: tile shape and plane chunks per level.

For every level of a workload it first times each compiled tile shape (rows
per wave x waves per workgroup) with the library's own HIP-event timing of
the sweep kernel and keeps the fastest; then, level by level, it times whole
runs (sweep plus the combine of plane chunks) for each plane-chunk count and
keeps the fastest.  The choice is remembered in a JSON cache keyed by the
device, the level shapes, the source count, the staging precision and the
launch kind.  Deterministic: a cached choice is reused as is."""
from __future__ import annotations

import json
import os

import torch

from .sweep import PlaneSweep

CANDIDATES = [(4, 4), (8, 4), (4, 8), (2, 8), (16, 4), (8, 2)]
CHUNK_CANDIDATES = [0, 1, 2, 3, 4, 6, 8]  # 0: the library's automatic count
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "psweep_tiles.json")


def _key(sweep: PlaneSweep, frames) -> str:
    props = torch.cuda.get_device_properties(sweep.device)
    lv = ";".join(f"{l.n_fronto}+{l.n_ground}w{l.window}d{l.downsample}c{tuple(l.crop)}" for l in sweep.settings.levels)
    sizes = ",".join(f"{f['ref'].shape[1]}x{f['ref'].shape[0]}" for f in frames)
    return (f"{props.gcnArchName}|{lv}|S{len(frames[0]['srcs'])}|st{sweep.cfg.storage}|"
            f"launch{sweep.cfg.launch}|{sizes}")


def _time(sweep, frames, outputs, reps):
    sweep.set_timing(True)
    best = float("inf")
    for _ in range(reps):
        sweep.run(frames, outputs)
        torch.cuda.synchronize()
        ms, n = sweep.sweep_kernel_ms()
        best = min(best, ms * n)
    sweep.set_timing(False)
    return best


def _run_ms(sweep, frames, outputs, reps):
    """Fastest whole run (every kernel of psweep_run), HIP events on the
    launch stream."""
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sweep.run(frames, outputs)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _apply(sweep, choice):
    for l, (r, w) in enumerate(choice["tiles"]):
        sweep.set_tile(l, r, w)
    for l, c in enumerate(choice.get("chunks", [0] * len(choice["tiles"]))):
        sweep.set_chunks(l, c)


def tune(sweep: PlaneSweep, frames, outputs, reps: int = 5, cache_path: str | None = DEFAULT_CACHE,
         candidates=CANDIDATES, chunk_candidates=CHUNK_CANDIDATES) -> dict:
    """Pick a tile shape per level (one shape for all levels with the
    persistent launch), then a plane-chunk count per level.  Returns {"key":
    ..., "tiles": [[rows, waves], ...], "chunks": [...], "ms": ...} and
    applies it to `sweep`."""
    key = _key(sweep, frames)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    nl = len(sweep.settings.levels)
    if key in cache:
        choice = cache[key]
        _apply(sweep, choice)
        return choice
    persistent = sweep.cfg.launch == 1
    results = {}
    for cand in candidates:
        try:
            for l in range(nl):
                sweep.set_tile(l, *cand)
            results[cand] = _time(sweep, frames, outputs, reps)
        except Exception:   # shape not compiled for this window / source count
            results[cand] = float("inf")
    if persistent:
        best = min(results, key=results.get)
        tiles = [list(best)] * nl
        ms = results[best]
    else:
        # levels are launched one after another; per-level times come back in order
        tiles, ms = [], 0.0
        per_level = {}
        for cand in candidates:
            if results[cand] == float("inf"):
                continue
            for l in range(nl):
                sweep.set_tile(l, *cand)
            sweep.set_timing(True)
            sweep.run(frames, outputs)
            torch.cuda.synchronize()
            sweep.set_timing(False)
            per_level[cand] = _per_launch_ms(sweep)
        for l in range(nl):
            best = min(per_level, key=lambda c: per_level[c][l] if l < len(per_level[c]) else float("inf"))
            tiles.append(list(best))
            ms += per_level[best][l]
    for l, (r, w) in enumerate(tiles):
        sweep.set_tile(l, r, w)
    # plane chunks, level by level, on whole-run time (the combine of chunks
    # is a kernel of its own)
    chunks, chunk_ms = [], {}
    for l in range(nl):
        best_c, best_t = 0, float("inf")
        for c in chunk_candidates:
            sweep.set_chunks(l, c)
            t = _run_ms(sweep, frames, outputs, reps)
            chunk_ms[f"level{l}:{c}"] = t
            if t < best_t:
                best_c, best_t = c, t
        sweep.set_chunks(l, best_c)
        chunks.append(best_c)
    choice = {"key": key, "tiles": tiles, "chunks": chunks, "ms": ms, "run_ms": min(chunk_ms.values()),
              "candidates": {f"{r}x{w}": v for (r, w), v in results.items()}, "chunk_candidates": chunk_ms}
    if cache_path:
        cache[key] = choice
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice


def _per_launch_ms(sweep):
    """Per-launch sweep durations of the last timed run, in launch order."""
    from . import psweep as P
    return P.psweep_sweep_kernel_times(sweep.ctx)
