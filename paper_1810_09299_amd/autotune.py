"""Launch-configuration tuner for batches and single cases.

Times a short run of the real workload for every candidate (tile height,
persistent grid or one workgroup per tile, case order) and keeps the fastest.
Every candidate gives bit-identical results, so tuning never changes answers.
"""
from __future__ import annotations

import itertools


def _events():
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    return a, b


def time_batch(batch, chunk: int, steps: int) -> float:
    """Milliseconds per step of `steps` steps of a batch whose cases run long enough."""
    import torch
    batch.run(chunk)
    batch.sync()
    a, b = _events()
    a.record(batch.stream)
    for _ in range(max(1, steps // chunk)):
        batch.run(chunk)
    b.record(batch.stream)
    batch.sync()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (max(1, steps // chunk) * chunk)


def tune_batch(make_batch, tiles=(8, 16, 4), persistent=(0, 1), schedules=(1,), chunk: int = 100,
               steps: int = 300):
    """make_batch() -> a Batch with its cases admitted.  Returns (best config, timings)."""
    timings = {}
    b = make_batch()
    for tr, pe, sc in itertools.product(tiles, persistent, schedules):
        b.set_config(tr, pe, sc)
        timings[(tr, pe, sc)] = time_batch(b, chunk, steps)
    b.close()
    best = min(timings, key=timings.get)
    return best, timings


def tune_case(make_case, tiles=(2, 4, 8, 16), steps: int = 200) -> int:
    """Tile height with the shortest step for a single case."""
    import torch
    best = None
    for tr in tiles:
        c = make_case()
        c.set_tile(tr)
        c.step(20)
        torch.cuda.synchronize()
        a, b = _events()
        a.record(c.stream)
        c.step(steps)
        b.record(c.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        if best is None or ms < best[1]:
            best = (tr, ms)
        c.close()
    return best[0]
