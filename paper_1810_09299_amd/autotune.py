"""Launch-configuration tuner for batches and single cases.

Times a short run of the real workload for every candidate -- tile height,
persistent grid or one workgroup per tile, the case-to-workgroup schedule
(case order, and whether each XCD takes strided or contiguous bands of a
case), and the number of contiguous tile bands each case is cut into for the
XCDs -- and keeps the fastest; the few fastest are timed a second time
and keep their better timing, so that one noisy run does not decide.  Every
candidate gives bit-identical results, so tuning never changes answers.
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


def tune_batch(make_batch, tiles=(8, 16, 4), persistent=(0, 1), schedules=(1, 0, 3, 2), bands=(16, 8, 32),
               chunk: int = 100, steps: int = 200, retime: int = 4):
    """make_batch() -> a Batch with its cases admitted.  Returns (best config
    (tile_r, persistent, schedule, bands), {config: ms per step})."""
    timings = {}
    b = make_batch()
    for tr, pe, sc, nb in itertools.product(tiles, persistent, schedules, bands):
        b.set_config(tr, pe, sc, nb)
        timings[(tr, pe, sc, nb)] = time_batch(b, chunk, steps)
    for cfg in sorted(timings, key=timings.get)[:retime]:
        b.set_config(*cfg)
        timings[cfg] = min(timings[cfg], time_batch(b, chunk, steps))
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
