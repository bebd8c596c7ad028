"""Continuous batching of axisymmetric solves (requests of different grid sizes
and step counts arriving over time).

A request is admitted as soon as it has arrived and the batch has a free slot
and a pool block large enough for its state (admission by HBM footprint, in
arrival order); admitted requests advance together, one fused launch per step
for all of them, in chunks of `chunk` steps replayed from a hipGraph; a request
that reaches its step count is read back (fields and diagnostics at its final
time) and released, freeing its slot and memory for the next arrivals.
Latency = completion time - arrival time.

The GPU is never drained: the next chunk is enqueued before the requests that
finished in the previous one are read back (the library reads a finished case
on a second stream, after its own last step only), and a new request is
initialised on that second stream while the queued chunk runs.  A request
whose state can never fit the pool is rejected when it arrives.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import abi, inputs
from .batch import Batch


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of serving
    spec: inputs.CaseSpec
    steps: int
    admitted: float = math.nan
    finished: float = math.nan
    diag: dict | None = None
    fields: dict | None = None
    rejected: bool = False

    @property
    def work(self) -> int:
        return self.spec.nr * self.spec.nz * self.steps


def sweep_requests(n: int, base_seed: int = 1810):
    """The first n requests of the seeded serving sweep (arrival times unset)."""
    out = []
    for i in range(n):
        s = inputs.serving_request(i, base_seed)
        out.append(Request(rid=i, arrival=0.0, spec=s, steps=s.steps))
    return out


def poisson_arrivals(reqs, rate_per_s: float, seed: int = 7):
    """Assign Poisson arrival times (exponential gaps from SplitMix64 deviates)."""
    u = 0.5 * (inputs.uniform_pm1(seed, np.arange(len(reqs), dtype=np.uint64)) + 1.0)
    gaps = -np.log1p(-np.minimum(u, 1 - 1e-16)) / rate_per_s
    t = np.cumsum(gaps)
    for r, a in zip(reqs, t):
        r.arrival = float(a)
    return reqs


def serve(reqs, pool_bytes: int, max_cases: int = 256, precision: str = "fp32", chunk: int = 200,
          keep_fields: bool = False, log=None):
    """Run the requests to completion; returns (requests, summary dict)."""
    import torch
    batch = Batch(pool_bytes=pool_bytes, max_cases=max_cases, precision=precision)
    pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
    running = {}            # slot -> request, admitted and not yet read back
    finished_prev = []      # slots whose last step is in a chunk enqueued before the latest one
    t0 = time.perf_counter()
    busy_chunks = 0
    max_running = 0
    while pending or running:
        now = time.perf_counter() - t0
        # admission, in arrival order, while slots and pool memory allow
        while pending and pending[0].arrival <= now:
            r = pending[0]
            try:
                slot = batch.admit(r.spec, r.steps)
            except abi.LbmAxiError as e:
                if e.code != abi.LBM_AXI_ENOMEM:
                    raise
                pending.popleft()           # larger than the whole pool: never admissible
                r.rejected = True
                r.finished = time.perf_counter() - t0
                continue
            if slot is None:
                break
            pending.popleft()
            r.admitted = time.perf_counter() - t0
            running[slot] = r
        max_running = max(max_running, len(running))
        active = batch.info()["running"] > 0
        if active:
            batch.run(chunk)
            busy_chunks += 1
        # read back what finished before that chunk: the GPU works on it meanwhile
        for slot in finished_prev:
            r = running.pop(slot)
            fields, diag, rc = batch.moments(slot, fields=keep_fields)
            r.finished = time.perf_counter() - t0
            r.diag = diag
            r.fields = fields if keep_fields else None
            batch.release(slot)
            if log:
                log(r)
        finished_prev = batch.poll()
        if not active and not finished_prev and pending:
            wait = pending[0].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
    batch.sync()
    makespan = time.perf_counter() - t0
    batch.close()
    torch.cuda.synchronize()
    done = [r for r in reqs if not r.rejected]
    lat = np.array([r.finished - r.arrival for r in done]) if done else np.array([math.nan])
    work = sum(r.work for r in done)
    return reqs, {
        "requests": len(reqs),
        "rejected": len(reqs) - len(done),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "aggregate_mlups": work / makespan / 1e6,
        "makespan_s": makespan,
        "lattice_updates": work,
        "max_running": max_running,
        "chunks": busy_chunks,
        "nonfinite": int(sum(1 for r in done if r.diag and r.diag["nonfinite"])),
    }


def saturated_throughput(reqs, pool_bytes: int, precision: str = "fp32", chunk: int = 200):
    """Closed-loop aggregate lattice updates per second of the mix: every request
    available at t = 0, the batch kept as full as the pool allows."""
    for r in reqs:
        r.arrival = 0.0
    _, summ = serve(reqs, pool_bytes, precision=precision, chunk=chunk)
    return summ["aggregate_mlups"] * 1e6


def load_sweep(n: int = 128, load: float = 0.8, pool_bytes: int = 4 << 30, precision: str = "fp32",
               chunk: int = 200, base_seed: int = 1810):
    """Serving sweep at `load` x the saturated throughput of the same mix."""
    cal = sweep_requests(n, base_seed)
    C = saturated_throughput(cal, pool_bytes, precision, chunk)
    reqs = sweep_requests(n, base_seed)
    mean_work = float(np.mean([r.work for r in reqs]))
    rate = load * C / mean_work
    poisson_arrivals(reqs, rate)
    reqs, summ = serve(reqs, pool_bytes, precision=precision, chunk=chunk)
    summ.update({"load": load, "saturated_mlups": C / 1e6, "arrival_rate_per_s": rate,
                 "offered_mlups": rate * mean_work / 1e6,
                 "pool_bytes": pool_bytes, "chunk_steps": chunk, "precision": precision})
    return reqs, summ
