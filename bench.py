#!/usr/bin/env python3
"""Throughput of the axisymmetric Allen-Cahn MRT lattice Boltzmann step on one MI355X.

Workload: the viscous-droplet-oscillation case, Nr x Nz = 256 x 512 (r x z),
periodic in z, density ratio 1000, synthetic seeded initial field.  One step =
one fused collide-and-stream update of both populations at every node (one
kernel launch).  Prints one JSON line:

  value         whole-job lattice updates per second, in MLUPS (inputs resident
                in HBM; the timed region holds exactly --steps steps)
  roofline      the step kernel against MI355X's 8 TB/s HBM: algorithmic bytes
                per launch (nodes x bytes per lattice update) over the mean
                launch duration, timed with HIP events on the library's stream
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per lattice update: 18 populations read + written,
# 3 previous-step values (phi, u_z, u_r) read + written
BYTES_PER_LU = {"fp64": 18 * 8 * 2 + 3 * 8 * 2, "fp32": 18 * 4 * 2 + 3 * 4 * 2}
WORKLOAD = "oscillating_droplet"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_1810_09299_amd/csrc/lbm_axi.hip", "paper_1810_09299_amd/csrc/axi_device.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_oscillating_droplet_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    rec = d.get(precision)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_steps(case, steps, warmup):
    """(wall seconds, event milliseconds) of exactly `steps` steps.  The HIP
    events are recorded on the stream the library launches on, bracketing
    the timed region, which holds one step-kernel launch per step."""
    import torch
    case.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(case.stream)
    case.step(steps)
    end.record(case.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(end)


def autotune_tile(spec, precision, trials=200):
    """Pick the tile height (rows per workgroup) with the shortest step."""
    from paper_1810_09299_amd.case import AxiCase
    best = None
    for tr in (2, 4, 8, 16):
        c = AxiCase(spec, precision=precision)
        c.set_tile(tr)
        _, dt = time_steps(c, trials, 20)
        if best is None or dt < best[1]:
            best = (tr, dt)
        c.close()
    return best[0]


def run_precision(spec, precision, steps, warmup, tile=None):
    from paper_1810_09299_amd.case import AxiCase
    tile = tile or autotune_tile(spec, precision)
    case = AxiCase(spec, precision=precision)
    case.set_tile(tile)
    dt, ev_ms = time_steps(case, steps, warmup)
    mean_ms = ev_ms / steps
    _, diag, rc = case.moments(fields=False)
    nodes = spec.nr * spec.nz
    bytes_launch = nodes * BYTES_PER_LU[precision]
    achieved = bytes_launch / (mean_ms * 1e-3) / 1e9
    return {
        "mlups": nodes * steps / dt / 1e6,
        "ms_per_step": dt / steps * 1e3,
        "kernel_ms_mean": mean_ms,
        "achieved_GBs": achieved,
        "bytes_per_launch": bytes_launch,
        "tile_rows": tile,
        "t_end": diag["t"],
        "umax_end": diag["umax"],
        "finite": rc == 0,
    }


def cpu_baseline(spec, steps=60):
    """The FP64 oracle (single-threaded C) on `steps` steps of the workload."""
    import oracle
    c = oracle.OracleCase(spec)
    c.step(2)
    t0 = time.perf_counter()
    c.step(steps)
    dt = time.perf_counter() - t0
    nodes = spec.nr * spec.nz
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the {spec.nr}x{spec.nz} oscillating droplet after 2 warm-up "
                      f"steps, single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="tile rows (0: autotune)")
    ap.add_argument("--only", action="store_true", help="skip the other precision")
    ap.add_argument("--cpu-steps", type=int, default=60)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent cases shard by case across GPUs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    from paper_1810_09299_amd import inputs

    spec = inputs.workload(WORKLOAD)
    main_res = run_precision(spec, args.precision, args.steps, args.warmup, args.tile)
    other = "fp32" if args.precision == "fp64" else "fp64"
    other_res = None if args.only else run_precision(spec, other, args.steps, args.warmup, args.tile)

    nodes = spec.nr * spec.nz
    traffic = measured_traffic(args.precision)
    line = {
        "metric": "MLUPS + % HBM roofline, FP64 vs FP32/FP16-store; p50/p99 batched-solve latency",
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD} {spec.nr}x{spec.nz} (nr x nz), periodic z, "
                               f"density ratio {spec.rho_l / spec.rho_g:g}, single case",
                   "nr": spec.nr, "nz": spec.nz, "nodes": nodes, "precision": args.precision,
                   "tile_rows": main_res["tile_rows"], "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "achieved": round(main_res["achieved_GBs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_res["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "step_kernel",
            "kernel_ms_mean": round(main_res["kernel_ms_mean"], 5),
            "bytes_per_launch": main_res["bytes_per_launch"],
        },
        "variants": {},
        "finite": main_res["finite"],
    }
    if other_res:
        line["variants"][other] = {"mlups": round(other_res["mlups"], 1),
                                   "achieved_GBs": round(other_res["achieved_GBs"], 1),
                                   "frac": round(other_res["achieved_GBs"] / HBM_PEAK_GBS, 4),
                                   "kernel_ms_mean": round(other_res["kernel_ms_mean"], 5),
                                   "tile_rows": other_res["tile_rows"]}
        line["finite"] = line["finite"] and other_res["finite"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
