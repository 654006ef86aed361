"""Autotuner of the raster kernels' launch settings (igs_set_launch_config).

Every candidate gives bit-identical results; only the time differs.  The tuner times a few
graph-replayed iterations of the caller's own fitter under each candidate, restores the fitter's
state after each trial, and leaves the fastest candidate set (the fitter's graph is re-captured
under it).  Candidates: one workgroup per tile or a persistent grid of 4, 5, 6 or 8 workgroups
per CU, each with and without the forward's candidate culling.  The single-pass fitting kernel
always runs one workgroup per tile, so for a single-pass fitter only the culling switch is timed.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _native as nat

Config = Tuple[int, int, int]   # (persistent, wgs_per_cu, fwd_cull)

DEFAULT_CANDIDATES: Tuple[Config, ...] = (
    (0, 0, 1), (0, 0, 0), (1, 4, 1), (1, 5, 1), (1, 6, 1), (1, 8, 1), (1, 0, 1),
)
SINGLE_PASS_CANDIDATES: Tuple[Config, ...] = ((0, 0, 1), (0, 0, 0))


def set_config(cfg: Config) -> None:
    nat.igs_set_launch_config(*cfg)


def current_config() -> Config:
    return nat.igs_get_launch_config().as_tuple()


def _time_fitter(fitter, iters: int, warmup: int) -> float:
    """Seconds per iteration over `iters` graph replays of a freshly captured iteration."""
    fitter.graph = None
    fitter.capture()
    for _ in range(warmup):
        fitter.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        fitter.step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters


def autotune(fitter, candidates: Optional[Sequence[Config]] = None, iters: int = 5,
             warmup: int = 2) -> Tuple[Config, Dict[Config, float]]:
    """Times `fitter` (a PlainFitter or BatchFitter whose pair buffer is already sized) under each
    candidate; sets and returns the fastest, with every candidate's seconds per iteration.  The
    fitter's parameters, moments and step count are restored after every trial."""
    if candidates is None:
        candidates = (SINGLE_PASS_CANDIDATES if getattr(fitter, "single_pass", False)
                      else DEFAULT_CANDIDATES)
    cands: List[Config] = list(candidates)
    state = fitter.snapshot()
    times: Dict[Config, float] = {}
    for c in cands:
        set_config(c)
        times[c] = _time_fitter(fitter, iters, warmup)
        fitter.restore(state)
    best = min(times, key=times.get)
    set_config(best)
    fitter.graph = None
    fitter.restore(state)
    return best, times
