"""Autotuner of the raster kernels' launch settings (igs_set_launch_config).

A setting is (persistent, wgs_per_cu, fwd_cull, fwd_batch, k_unroll): tile scheduling (one
workgroup per tile, or a persistent grid of resident workgroups pulling tiles from the shared
queue, which for a batch is ordered largest hit set first), the forward's candidate culling, the
number of candidates the forward stages in LDS at a time, and the length of its register-resident
top-K list.  Every setting gives bit-identical results; only the time differs.  The tile size is
not among them: it is part of the definition of the hit sets S_j (16 x 16, Sec. 4.1).

After one untimed warm-up trial, the tuner times a few graph-replayed iterations of the caller's
own fitter per candidate, by coordinate descent: first the scheduling and culling with the default blocking, then the LDS
batch size under the best scheduling, then the list length under both.  It restores the fitter's
state after each trial and gives the fitter the fastest setting as its own launch settings (also
set on the calling thread; the fitter's graph is re-captured under it).
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _native as nat

Config = Tuple[int, int, int, int, int]   # (persistent, wgs_per_cu, fwd_cull, fwd_batch, k_unroll)

DEFAULT: Config = (0, 0, 1, 192, 0)
# scheduling and culling: one workgroup per tile, or persistent grids of 4, 5, 6, 8 or as many
# workgroups per CU as fit
SCHEDULES: Tuple[Tuple[int, int, int], ...] = (
    (0, 0, 1), (0, 0, 0), (1, 4, 1), (1, 5, 1), (1, 6, 1), (1, 8, 1), (1, 0, 1),
)
SINGLE_PASS_SCHEDULES: Tuple[Tuple[int, int, int], ...] = ((0, 0, 1), (0, 0, 0), (1, 0, 1))
FWD_BATCHES: Tuple[int, ...] = (128, 192, 256)
KT_COMPILED: Tuple[int, ...] = (1, 2, 4, 8, 10, 16, 32)


def set_config(cfg: Sequence[int]) -> None:
    nat.igs_set_launch_config(*cfg)


def current_config() -> Config:
    return nat.igs_get_launch_config().as_tuple()


def list_lengths(K: int) -> List[int]:
    """The compiled list lengths a setting can select for top-K: the smallest one >= K (k_unroll
    0) and the next longer one."""
    longer = [kt for kt in KT_COMPILED if kt >= K]
    return [0] + longer[1:2]


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
    candidate and gives it the fastest; returns that setting and every trial's seconds per
    iteration.  Without explicit candidates the search is the coordinate descent of the module
    notes.  The fitter's parameters, moments and step count are restored after every trial."""
    state = fitter.snapshot()
    times: Dict[Config, float] = {}
    # one untimed trial first: the first timed one would otherwise also pay for the device and
    # its caches warming up
    fitter.launch_config = tuple(candidates[0]) if candidates is not None else DEFAULT
    _time_fitter(fitter, iters, warmup)
    fitter.restore(state)

    def trial(c: Config) -> float:
        if c not in times:
            fitter.launch_config = c
            times[c] = _time_fitter(fitter, iters, warmup)
            fitter.restore(state)
        return times[c]

    if candidates is not None:
        for c in candidates:
            trial(tuple(c))
        best = min(times, key=times.get)
    else:
        sched = (SINGLE_PASS_SCHEDULES if getattr(fitter, "single_pass", False) else SCHEDULES)
        best = min((s + DEFAULT[3:] for s in sched), key=trial)
        best = min((best[:3] + (fb, best[4]) for fb in FWD_BATCHES), key=trial)
        best = min((best[:4] + (ku,) for ku in list_lengths(fitter.K)), key=trial)
    fitter.launch_config = best   # the fitter keeps its choice whatever other callers set
    set_config(best)
    fitter.graph = None
    fitter.restore(state)
    return best, times
