#!/usr/bin/env python3
"""Throughput of the axisymmetric Allen-Cahn MRT lattice Boltzmann step on one MI355X.

Workload: the viscous-droplet-oscillation case, Nr x Nz = 256 x 512 (r x z),
periodic in z, density ratio 1000, synthetic seeded initial fields; solved as a
batch of --cases independent cases (jitter seeds 1..B; 64 cases hold 1.6 GB in
FP32, six times the 256 MB Infinity Cache), every step one fused
collide-and-stream launch over all of them.  The steps run as hipGraph
replays of chunks of min(100, --steps) steps plus a directly launched tail
(step_plan); warm-up runs --warmup steps the same way, and the graphs the
timed runs replay are captured before the timed region.  Prints one JSON line:

  value         whole-job lattice updates per second, MLUPS (states resident in
                HBM; the timed region holds exactly --steps steps of the batch)
  roofline      the batched step kernel against MI355X's 8 TB/s HBM:
                algorithmic bytes per launch (cases x nodes x bytes per lattice
                update) over the mean launch duration, from HIP events on the
                batch's stream around the timed region
  variants      the batch in the other storage precisions; the batch with the
                SRT and non-orthogonal MRT collision forms in every precision;
                FP16-deviation storage with stochastic g rounding; single case
                FP64, FP32 and FP16 storage (the plain path)
  errors        FP32, FP16 (both g roundings) vs FP64 after 1000 steps of one case
  serving       continuous batching of the seeded request sweep at 80 % load:
                p50 / p99 latency and aggregate MLUPS (512 requests in FP32
                storage; serving_fp16: the first 128 in FP16-deviation storage)
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload:
                one thread, and one process per core on up to 16 cores (run
                before the GPU is touched)

roofline also carries copy_GBs, the bandwidth a plain device copy of 1 GiB
reaches on the same device (lbm_axi_device_copy, HIP events), and
frac_of_copy = achieved / copy_GBs: the published 8 TB/s is not reachable by
any access pattern, a plain copy sets the practical ceiling.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per lattice update, read + write: 18 populations and 3
# aux values (phi, u_z, u_r) of the storage type; FP16-deviation storage: 18
# FP16 populations and FP32 aux.  (Its implementation keeps f_0 in FP32 for
# exact mass and so moves 100 B; the algorithmic count is the method's 96 B.)
BYTES_PER_LU = {"fp64": 18 * 8 * 2 + 3 * 8 * 2, "fp32": 18 * 4 * 2 + 3 * 4 * 2,
                "fp16": 18 * 2 * 2 + 3 * 4 * 2}
MOVED_BYTES_PER_LU = dict(BYTES_PER_LU, fp16=(4 + 8 * 2 + 9 * 2) * 2 + 3 * 4 * 2)
WORKLOAD = "oscillating_droplet"
CHUNK = 100
CASES = 64
CPU_POOL_MAX = 16        # worker processes of the all-core CPU baseline
METRIC = "MLUPS + % HBM roofline, FP64 vs FP32/FP16-store; p50/p99 batched-solve latency"


def note(msg: str) -> None:
    """Progress of the run on stderr (the JSON line goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_1810_09299_amd/csrc/lbm_axi.hip", "paper_1810_09299_amd/csrc/lbm_axi_batch.hip",
                "paper_1810_09299_amd/csrc/axi_device.hpp", "paper_1810_09299_amd/csrc/axi_half.hpp",
                "paper_1810_09299_amd/csrc/case_internal.hpp", "paper_1810_09299_amd/build.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_plan(steps: int, chunk: int = CHUNK) -> list:
    """Run lengths adding up to exactly `steps`: runs of min(chunk, steps)
    steps (each a hipGraph replay), then the remainder (launched directly)."""
    if steps <= 0:
        return []
    c = min(chunk, steps)
    plan = [c] * (steps // c)
    if steps % c:
        plan.append(steps % c)
    return plan


def measured_traffic(precision: str, config, cases: int) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source with the same number of cases and
    launch configuration (tile rows, persistent, schedule, bands); else None."""
    path = os.path.join(ROOT, "profiles", "batch_step_kernel_oscillating_droplet_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    key = f"{cases}/{config['tile_rows']}/{config['persistent']}/{config['schedule']}/{config['bands']}"
    rec = d.get(precision, {}).get(key)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def batch_specs(n):
    from paper_1810_09299_amd import inputs
    out = []
    for q in range(n):
        s = inputs.workload(WORKLOAD)
        if q:
            s = inputs.oscillating_droplet(nr=s.nr, nz=s.nz, R0=60.0, seed=1 + q, zc=256.0, W=4.0,
                                           ratio=1000.0, sigma=1e-3, mobility=0.05, z_periodic=True)
        out.append(s)
    return out


def make_batch(specs, precision):
    from paper_1810_09299_amd.batch import Batch
    pool = Batch.pool_for(specs, precision)
    b = Batch(pool_bytes=pool, max_cases=len(specs), precision=precision)
    for s in specs:
        assert b.admit(s, 10 ** 12) is not None
    return b


def run_batch(specs, precision, steps, warmup, config=None):
    """Exactly `steps` timed steps of the batch after `warmup` untimed ones."""
    import torch
    from paper_1810_09299_amd import autotune
    if config is None:
        # cases of one size: both case orders give the same work list (the
        # band order, schedule bit 1, still matters)
        same = len({(q.nr, q.nz) for q in specs}) == 1
        config, _ = autotune.tune_batch(lambda: make_batch(specs, precision),
                                        schedules=(1, 3) if same else (1, 0, 3, 2))
    b = make_batch(specs, precision)
    b.set_config(*config)
    for m in step_plan(warmup):
        b.run(m)
    timed = step_plan(steps)
    for m in sorted(set(timed)):
        b.prepare(m)            # capture the replayed graphs outside the timed region
    b.sync()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(b.stream)
    for m in timed:
        b.run(m)
    end.record(b.stream)
    b.sync()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(end)
    k = sum(timed)
    diags = [b.moments(s, fields=False) for s in range(len(specs))]
    finite = all(d[2] == 0 for d in diags)
    b.close()
    nodes = sum(s.nr * s.nz for s in specs)
    kernel_ms = ev_ms / k
    note(f"batch {len(specs)} x {specs[0].nr}x{specs[0].nz} {precision} {specs[0].collision} config {config}: "
         f"{kernel_ms * 1e3:.2f} us per step, {nodes * k / wall / 1e6:.0f} MLUPS")
    bytes_launch = nodes * BYTES_PER_LU[precision]
    return {"mlups": nodes * k / wall / 1e6, "ms_per_step": wall / k * 1e3, "kernel_ms": kernel_ms,
            "achieved_GBs": bytes_launch / (kernel_ms * 1e-3) / 1e9, "bytes_per_launch": bytes_launch,
            "steps": k, "config": {"tile_rows": config[0], "persistent": config[1], "schedule": config[2],
                                   "bands": config[3]},
            "finite": finite, "t_final": diags[0][1]["t"]}


def copy_peak(nbytes: int = 1 << 30, reps: int = 20) -> float:
    """GB/s of the library's plain device copy of nbytes (read + write
    counted), HIP events on the stream the copies are launched on."""
    import torch
    from paper_1810_09299_amd import abi
    src = torch.full((nbytes // 4,), 1.0, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        abi.lbm_axi_device_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        abi.lbm_axi_device_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / reps
    if not torch.equal(src, dst):
        raise RuntimeError("lbm_axi_device_copy produced a wrong copy")
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_single(spec, precision, steps, warmup):
    import torch
    from paper_1810_09299_amd import autotune
    from paper_1810_09299_amd.case import AxiCase
    tile = autotune.tune_case(lambda: AxiCase(spec, precision=precision))
    c = AxiCase(spec, precision=precision)
    c.set_tile(tile)
    c.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(c.stream)
    c.step(steps)
    end.record(c.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = spec.nr * spec.nz
    kernel_ms = start.elapsed_time(end) / steps
    return {"mlups": nodes * steps / wall / 1e6, "kernel_ms": kernel_ms,
            "achieved_GBs": nodes * BYTES_PER_LU[precision] / (kernel_ms * 1e-3) / 1e9, "tile_rows": tile}


def precision_errors(spec, precision, steps=1000):
    """Fields of `precision` against the FP64 GPU path after `steps` steps."""
    import numpy as np
    from paper_1810_09299_amd.case import AxiCase
    a = AxiCase(spec, precision="fp64")
    b = AxiCase(spec, precision=precision)
    _, d0, _ = b.moments(fields=False)
    a.step(steps)
    b.step(steps)
    ma, da, _ = a.moments()
    mb, db, _ = b.moments()
    un = max(np.abs(ma["uz"]).max(), np.abs(ma["ur"]).max())
    return {"steps": steps,
            "phi_max_abs": float(np.abs(ma["phi"] - mb["phi"]).max()),
            "u_max_rel": float(max(np.abs(ma["uz"] - mb["uz"]).max(), np.abs(ma["ur"] - mb["ur"]).max()) / un),
            "phase_mass_rel_vs_fp64": float(abs(db["phase_mass"] / da["phase_mass"] - 1.0)),
            "phase_mass_drift": float(abs(db["phase_mass"] / d0["phase_mass"] - 1.0)),
            "reference": "FP64 GPU path (oracle parity <= 1e-12 per step)"}


def laplace_errors(precision, steps=2000):
    """Static droplet at the paper's density scale: Laplace pressure jump of
    `precision` against the FP64 GPU path."""
    from paper_1810_09299_amd import inputs
    from paper_1810_09299_amd.case import AxiCase
    spec = inputs.workload("static_droplet")
    dp = {}
    for prec in ("fp64", precision):
        c = AxiCase(spec, precision=prec)
        c.step(steps)
        dp[prec] = c.moments(fields=False)[1]["dp"]
    return {"workload": "static_droplet 64x128, density ratio 1000", "steps": steps, "dp_fp64": dp["fp64"],
            f"dp_{precision}": dp[precision], "dp_rel": abs(dp[precision] / dp["fp64"] - 1.0)}


def _oracle_sample(steps: int):
    """(lattice updates, start, end) of `steps` oracle steps of the workload
    after 2 warm-up steps (perf_counter times, comparable across processes)."""
    import oracle
    from paper_1810_09299_amd import inputs
    spec = inputs.workload(WORKLOAD)
    c = oracle.OracleCase(spec)
    c.step(2)
    t0 = time.perf_counter()
    c.step(steps)
    t1 = time.perf_counter()
    return spec.nr * spec.nz * steps, t0, t1


def cpu_baseline(steps_single=400, steps_each=150):
    """The FP64 oracle (plain single-threaded C, as it stands) on a bounded
    sample of the workload: one thread, then one process per core (up to
    CPU_POOL_MAX), each advancing its own copy of the case.  Must run before
    the GPU is initialised (the pool forks)."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    host_cores = os.cpu_count()
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else host_cores
    nproc = max(1, min(CPU_POOL_MAX, avail))
    lu, t0, t1 = _oracle_sample(steps_single)
    single = lu / (t1 - t0) / 1e6
    note(f"cpu baseline: one thread {single:.2f} MLUPS; now {nproc} processes")
    with mp.get_context("fork").Pool(nproc) as pool:
        res = pool.map(_oracle_sample, [steps_each] * nproc)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    allcore = sum(r[0] for r in res) / wall / 1e6
    return {"value": round(allcore, 3), "unit": "MLUPS", "cores": nproc, "kind": "oracle",
            "single_thread_mlups": round(single, 3), "all_core_mlups": round(allcore, 3),
            "host_cores": host_cores, "cores_available": avail,
            "sample": f"FP64 oracle on the 256x512 oscillating droplet after 2 warm-up steps: "
                      f"{steps_single} steps on one thread ({t1 - t0:.1f} s); then {nproc} processes, "
                      f"one per core, {steps_each} steps each of their own copy ({wall:.1f} s wall)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cases", type=int, default=CASES)
    ap.add_argument("--precision", default="fp32", choices=("fp64", "fp32", "fp16"))
    ap.add_argument("--tile", type=int, default=0, help="tile rows (0: autotune)")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--bands", type=int, default=16, help="tile bands per case (with --tile)")
    ap.add_argument("--schedule", type=int, default=1, help="case order (with --tile)")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the FP32 serving sweep (the sweep's full 512 by default)")
    ap.add_argument("--serving-requests-fp16", type=int, default=128,
                    help="requests of the same sweep in FP16-deviation storage")
    ap.add_argument("--fp16-stochastic", action="store_true",
                    help="FP16-deviation storage with stochastic g rounding (with --precision fp16)")
    ap.add_argument("--no-extras", action="store_true", help="only the primary measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=400)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(cases are independent and would shard by case across GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    # the CPU baseline forks its worker pool: before anything initialises the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_steps)
    import torch
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    from paper_1810_09299_amd import inputs

    specs = batch_specs(args.cases)
    stochastic = args.fp16_stochastic and args.precision == "fp16"
    for s in specs:
        s.fp16_stochastic = stochastic
    config = (args.tile, args.persistent, args.schedule, args.bands) if args.tile else None
    main_res = run_batch(specs, args.precision, args.steps, args.warmup, config)
    copy_gbs = copy_peak()
    spec = specs[0]
    nodes = spec.nr * spec.nz
    line = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": main_res["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD} {spec.nr}x{spec.nz} (nr x nz), periodic z, density ratio "
                               f"{spec.rho_l / spec.rho_g:g}; batched solve of {args.cases} independent cases",
                   "nr": spec.nr, "nz": spec.nz, "cases": args.cases, "nodes": nodes * args.cases,
                   "storage": args.precision, **({"g_rounding": "stochastic"} if stochastic else {}),
                   **main_res["config"], "chunk_steps": min(CHUNK, args.steps),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(main_res["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(main_res["achieved_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": (None if stochastic else
                                 measured_traffic(args.precision, main_res["config"], args.cases)),
                     "kernel": "batch_step_kernel",
                     "kernel_ms_mean": round(main_res["kernel_ms"], 5),
                     "bytes_per_launch": main_res["bytes_per_launch"],
                     "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(main_res["achieved_GBs"] / copy_gbs, 4)},
        "finite": main_res["finite"],
    }
    if not args.no_extras:
        line["variants"] = {}
        tuned = {args.precision: tuple(main_res["config"].values())}
        for other in ("fp64", "fp32", "fp16"):
            if other == args.precision:
                continue
            ob = run_batch(specs, other, args.steps, args.warmup)
            tuned[other] = tuple(ob["config"].values())
            line["variants"][f"batch_{other}"] = {
                "mlups": round(ob["mlups"], 1), "frac": round(ob["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "frac_of_copy": round(ob["achieved_GBs"] / copy_gbs, 4),
                "kernel_ms_mean": round(ob["kernel_ms"], 5), "bytes_per_lu": BYTES_PER_LU[other],
                "moved_bytes_per_lu": MOVED_BYTES_PER_LU[other], **ob["config"]}
        # the same batch at a quarter of the cases (411 MB in FP32), launch
        # configuration of the full batch
        if args.cases >= 32:
            qs = batch_specs(args.cases // 4)
            ob = run_batch(qs, args.precision, args.steps, args.warmup, tuple(main_res["config"].values()))
            line["variants"][f"batch_{args.precision}_{args.cases // 4}cases"] = {
                "mlups": round(ob["mlups"], 1), "frac": round(ob["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "kernel_ms_mean": round(ob["kernel_ms"], 5),
                "us_per_mlu": round(ob["kernel_ms"] * 1e3 / (sum(q.nr * q.nz for q in qs) / 1e6), 4),
                "cases": args.cases // 4, **ob["config"]}
            line["roofline"]["us_per_mlu"] = round(main_res["kernel_ms"] * 1e3 / (nodes * args.cases / 1e6), 4)
        # the other collision forms on the same batch, each precision's launch configuration
        for form in ("srt", "nmrt"):
            fspecs = batch_specs(args.cases)
            for fs in fspecs:
                fs.collision = form
            for prec in ("fp64", "fp32", "fp16"):
                ob = run_batch(fspecs, prec, min(args.steps, 500), args.warmup, tuned[prec])
                line["variants"][f"batch_{prec}_{form}"] = {
                    "mlups": round(ob["mlups"], 1), "frac": round(ob["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "kernel_ms_mean": round(ob["kernel_ms"], 5), "collision": form, **ob["config"]}
        # FP16-deviation storage with stochastic g rounding, FP16's launch configuration
        sspecs = batch_specs(args.cases)
        for fs in sspecs:
            fs.fp16_stochastic = True
        ob = run_batch(sspecs, "fp16", min(args.steps, 500), args.warmup, tuned["fp16"])
        line["variants"]["batch_fp16_stochastic"] = {
            "mlups": round(ob["mlups"], 1), "frac": round(ob["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "kernel_ms_mean": round(ob["kernel_ms"], 5), "g_rounding": "stochastic", **ob["config"]}
        for prec in ("fp64", "fp32", "fp16"):
            sr = run_single(spec, prec, args.steps, args.warmup)
            line["variants"][f"single_{prec}"] = {
                "mlups": round(sr["mlups"], 1), "frac": round(sr["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "kernel_ms_mean": round(sr["kernel_ms"], 5), "tile_rows": sr["tile_rows"]}
        note("single cases done; precision errors next")
        line["errors"] = {"fp32_vs_fp64": precision_errors(spec, "fp32"),
                          "fp16_vs_fp64": precision_errors(spec, "fp16"),
                          "fp16_stochastic_vs_fp64": precision_errors(
                              dataclasses.replace(spec, fp16_stochastic=True), "fp16"),
                          "fp16_laplace": laplace_errors("fp16")}
        from paper_1810_09299_amd import serving
        for prec, key, n in (("fp32", "serving", args.serving_requests),
                             ("fp16", "serving_fp16", args.serving_requests_fp16)):
            if n > 0:
                note(f"serving sweep: {n} requests, {prec}")
                _, summ = serving.load_sweep(n=n, load=0.8, precision=prec)
                line[key] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
