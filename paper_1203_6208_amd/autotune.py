"""Tile-size autotuner of the batched boxes.

The batched library stores every box's real-space matrix in square tiles of
32 or 64 beads.  Small boxes waste less padding and give more workgroups with
32-bead tiles; large boxes read longer rows with 64-bead tiles.  Which one is
faster for a given ensemble is measured, not modelled: ``tune_batch`` creates
the batch once per candidate, replays the captured step a few times and keeps
the fastest.  Results are cached per ensemble signature for the process.
"""
from __future__ import annotations

import hashlib

import torch

from . import rpy

CANDIDATES = (32, 64)
_cache: dict = {}


def signature(workloads, bp: rpy.BdParams, lowp: str) -> str:
    """Key of an ensemble + step configuration (box sizes, chain layout,
    geometry, Chebyshev order, precision)."""
    h = hashlib.sha1()
    for w in workloads:
        h.update(f"{w.n},{w.bpc},{w.L:.12g},{w.a:.12g},{w.alpha:.12g},{w.rc:.12g};".encode())
    h.update(f"{bp.n_cheb},{bp.bounds_rule},{bp.prec},{lowp}".encode())
    return h.hexdigest()


def time_candidate(workloads, bp: rpy.BdParams, lowp: str, tile_beads: int, positions,
                   steps: int = 3, warmup: int = 1, seed: int = 0) -> float:
    """Mean seconds per step of graph replays with the given tile size."""
    B = rpy.Batch(workloads, lowp=lowp, tile_beads=tile_beads)
    try:
        pos = B.pack(positions)
        B.run(pos, bp, seed=seed, step0=0, n_steps=warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.run(pos, bp, seed=seed, step0=warmup, n_steps=steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / steps
    finally:
        B.close()


def tune_batch(workloads, bp: rpy.BdParams, lowp: str = "f32", steps: int = 3,
               candidates=CANDIDATES, positions=None):
    """(best tile_beads, {tile_beads: seconds per step})."""
    key = signature(workloads, bp, lowp)
    if key in _cache:
        return _cache[key]
    if positions is None:
        positions = [w.positions() for w in workloads]
    times = {}
    for tb in candidates:
        times[tb] = time_candidate(workloads, bp, lowp, tb, positions, steps=steps)
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return best, times
