"""Autotuner of the batched boxes' step.

The batched library can run one ensemble step in several ways that give the
same values and differ only in time:

* ``tile_beads``: every box's real-space matrix is stored in square tiles of
  32 or 64 beads (fixed when the batch is created).  Small boxes waste less
  padding and give more workgroups with 32-bead tiles; large boxes read longer
  rows with 64-bead tiles.
* ``sf_place``: where the structure-factor workgroups of the tile-product
  launch sit -- spread evenly through it, so that their FP64 arithmetic
  overlaps the tile stream, or all at its front.
* ``tile_loads``: non-temporal tile loads (the tile arrays are larger than the
  caches) or ordinary, allocating ones.

Which combination is fastest for a given ensemble is measured, not modelled:
``tune_batch`` creates the batch once per tile size, sets every variant in
turn, replays the captured step a few times and keeps the fastest.  Results
are cached per ensemble signature for the process.
"""
from __future__ import annotations

import hashlib
import itertools
from dataclasses import dataclass

import torch

from . import rpy

TILES = (32, 64)
SF_PLACES = {"spread": rpy.SF_SPREAD, "front": rpy.SF_FRONT}
LOADS = {"stream": rpy.LOADS_STREAM, "cached": rpy.LOADS_CACHED}
_cache: dict = {}


@dataclass(frozen=True)
class Config:
    tile_beads: int = 64
    sf_place: str = "spread"
    tile_loads: str = "stream"

    def as_dict(self):
        return {"tile_beads": self.tile_beads, "sf_place": self.sf_place,
                "tile_loads": self.tile_loads}


def search_space(tiles=TILES, sf_places=tuple(SF_PLACES), loads=tuple(LOADS)):
    return [Config(t, s, l) for t, s, l in itertools.product(tiles, sf_places, loads)]


def make_batch(workloads, config: Config, lowp: str = "f32") -> rpy.Batch:
    """A batch over `workloads` set up as `config`."""
    B = rpy.Batch(workloads, lowp=lowp, tile_beads=config.tile_beads)
    B.set_variant(SF_PLACES[config.sf_place], LOADS[config.tile_loads])
    return B


def signature(workloads, bp: rpy.BdParams, lowp: str) -> str:
    """Key of an ensemble + step configuration (box sizes, chain layout,
    geometry, Chebyshev order, precision)."""
    h = hashlib.sha1()
    for w in workloads:
        h.update(f"{w.n},{w.bpc},{w.L:.12g},{w.a:.12g},{w.alpha:.12g},{w.rc:.12g};".encode())
    h.update(f"{bp.n_cheb},{bp.bounds_rule},{bp.prec},{lowp}".encode())
    return h.hexdigest()


def _time_replays(B: rpy.Batch, pos, bp, steps: int, warmup: int, seed: int) -> float:
    """Mean seconds per step of graph replays (the warm-up captures the graph)."""
    B.run(pos, bp, seed=seed, step0=0, n_steps=warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    B.run(pos, bp, seed=seed, step0=warmup, n_steps=steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def tune_batch(workloads, bp: rpy.BdParams, lowp: str = "f32", steps: int = 3,
               candidates=None, positions=None, warmup: int = 1, seed: int = 0):
    """(best Config, {Config: seconds per step}) over `candidates` (default:
    the whole search space)."""
    key = signature(workloads, bp, lowp)
    if candidates is None and key in _cache:
        return _cache[key]
    cands = search_space() if candidates is None else list(candidates)
    if positions is None:
        positions = [w.positions() for w in workloads]
    times = {}
    for tb in sorted({c.tile_beads for c in cands}):
        B = rpy.Batch(workloads, lowp=lowp, tile_beads=tb)
        try:
            pos0 = B.pack(positions)
            for c in (c for c in cands if c.tile_beads == tb):
                B.set_variant(SF_PLACES[c.sf_place], LOADS[c.tile_loads])
                pos = pos0.clone()
                times[c] = _time_replays(B, pos, bp, steps, warmup, seed)
        finally:
            B.close()
    best = min(times, key=times.get)
    if candidates is None:
        _cache[key] = (best, times)
    return best, times
