"""Chooses the launch schedule of a batch or a room by timing it on the
caller's own requests.

The schedule (search iterations per thread, width of the all-rounds scoring,
tree levels the traversal reads from LDS, rounds of the first all-rounds
scoring pass) changes no result: every hypothesis draws its samples from its
own Philox counters whichever thread runs it, every energy is summed in the
same order, and a node is the same bits from LDS or from global memory.  So the choice is a pure timing decision, made on
the device and workload that will use it.
"""

from __future__ import annotations

import ctypes
import time

import numpy as np

from . import SCHEDULE_FAST_WAVES, SCHEDULE_IPT, SCHEDULE_LDS_LEVELS, SCHEDULE_SCORE_WINDOWS, Result

DEFAULT = (4, 1, 8, 0)          # a room's default schedule
BATCH_DEFAULT = (4, 1, 8, 2)    # a batch's


def candidates(ipts=SCHEDULE_IPT, fast_waves=SCHEDULE_FAST_WAVES, lds_levels=SCHEDULE_LDS_LEVELS,
               windows=SCHEDULE_SCORE_WINDOWS, first=DEFAULT) -> list:
    """Every (iterations per thread, fast waves, LDS levels, score window)
    schedule, `first` (the default) first."""
    every = [(i, f, l, w) for i in ipts for f in fast_waves for l in lds_levels for w in windows]
    return ([first] if first in every else []) + [sc for sc in every if sc != first]


def pick(timings: dict, default=DEFAULT, margin: float = 0.02):
    """The schedule with the lowest median time.  The default stays unless
    another beats it by more than `margin` (a fraction of its time), so that
    timing noise does not move the choice; ties go to the earlier key."""
    if not timings:
        raise ValueError("no timings")
    med = {k: float(np.median(v)) for k, v in timings.items()}
    best = min(med, key=lambda k: (med[k], list(med).index(k)))
    if default in med and med[best] >= med[default] * (1.0 - margin):
        return default
    return best


def tune_batch(batch, reqs, schedules=None, reps: int = 5, warmup: int = 2, use_graph: bool = True):
    """Times `reqs` (the Batch.relocalise request list) under each schedule,
    sets the fastest on `batch` and returns (schedule, {schedule: [ms]}).
    Each time is the GPU time between events on the batch's stream around
    one queued batch (graph replays after the warm-up capture)."""
    import torch

    schedules = schedules or candidates(first=BATCH_DEFAULT)
    out = torch.empty(len(reqs) * ctypes.sizeof(Result), dtype=torch.uint8, device=batch.device)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    timings = {}
    for sc in schedules:
        batch.set_schedule(*sc)
        for _ in range(warmup):
            batch.relocalise_async(reqs, out, use_graph=use_graph)
        ms = []
        for _ in range(reps):
            ev0.record(batch.stream)
            batch.relocalise_async(reqs, out, use_graph=use_graph)
            ev1.record(batch.stream)
            ev1.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        timings[sc] = ms
    best = pick(timings, default=BATCH_DEFAULT)
    batch.set_schedule(*best)
    return best, timings


def tune_room(room, depth, rgb, K, schedules=None, reps: int = 7, warmup: int = 2, request_seed: int = 0):
    """Times one synchronous relocalisation of (depth, rgb, K) under each
    schedule (host wall clock, as a caller of the synchronous call sees it),
    sets the fastest on `room` and returns (schedule, {schedule: [ms]})."""
    schedules = schedules or candidates()
    timings = {}
    for sc in schedules:
        room.set_schedule(*sc)
        for _ in range(warmup):
            room.relocalise(depth, rgb, K, request_seed=request_seed)
        ms = []
        for _ in range(reps):
            t0 = time.perf_counter()
            room.relocalise(depth, rgb, K, request_seed=request_seed)
            ms.append((time.perf_counter() - t0) * 1e3)
        timings[sc] = ms
    best = pick(timings)
    room.set_schedule(*best)
    return best, timings
