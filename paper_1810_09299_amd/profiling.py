"""Helpers for the rocprofv3 summaries kept under profiles/.

  python3 -m paper_1810_09299_amd.profiling copy [GiB]
      a plain device-to-device copy of a known size (torch copy_), five times:
      the HBM byte counters (FETCH_SIZE, WRITE_SIZE) read on it calibrate the
      same counters read on the step kernels
  python3 -m paper_1810_09299_amd.profiling moments [nr nz reps precision]
      read-back of one oscillating-droplet case (default 256 x 512, 20 reads,
      fp32): the moments kernel and the three diagnostics passes, for a
      kernel trace of the read-back path
  python3 -m paper_1810_09299_amd.profiling stats <kernel_stats.csv>
      markdown table of a --kernel-trace --stats summary
  python3 -m paper_1810_09299_amd.profiling counter <counter_collection.csv> <kernel substring> <counter>
      mean per dispatch of one counter on the matching kernels
  python3 -m paper_1810_09299_amd.profiling traffic <kernel substring> <fetch.csv> <write.csv>
          <copy_fetch.csv> <copy_write.csv> <copy bytes>
      calibrated HBM bytes per dispatch of the kernel: each counter (KiB per
      dispatch) scaled by bytes / counter reading of the copy of known size
"""
from __future__ import annotations

import csv
import sys


def copy_probe(gib: float = 1.0, reps: int = 5) -> int:
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    nbytes = n * 4
    print(f"copied {nbytes} bytes x {reps}", flush=True)
    return nbytes


def moments_probe(nr: int = 256, nz: int = 512, reps: int = 20, precision: str = "fp32") -> dict:
    from . import inputs
    from .case import AxiCase
    spec = inputs.oscillating_droplet(nr=nr, nz=nz, R0=nr * 60.0 / 256.0, zc=nz / 2.0)
    c = AxiCase(spec, precision=precision)
    c.step(10)
    d = None
    for _ in range(reps):
        _, d, _ = c.moments(fields=False)
    print(f"moments of {nr}x{nz} {precision} read {reps} times: t = {d['t']}, R_eq = {d['R_eq']:.4f}", flush=True)
    return d


def kernel_stats(path: str):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                         "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                         "pct": float(r["Percentage"])})
    return rows


def stats_markdown(path: str, top: int = 12) -> str:
    out = ["| kernel | calls | avg (us) | min (us) | max (us) | % time |", "|---|---|---|---|---|---|"]
    for r in kernel_stats(path)[:top]:
        name = r["name"].replace("(anonymous namespace)::", "")
        name = name.split("(")[0] if "(" in name else name
        out.append(f"| `{name}` | {r['calls']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | {r['max_us']:.2f} | {r['pct']:.1f} |")
    return "\n".join(out)


def counter_mean(path: str, kernel_substring: str, counter: str):
    """(mean, count) of `counter` over dispatches whose kernel name contains the substring."""
    vals = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if kernel_substring not in r.get("Kernel_Name", ""):
                continue
            if r.get("Counter_Name") != counter:
                continue
            key = r.get("Dispatch_Id") or r.get("Correlation_Id")
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        return float("nan"), 0
    v = list(vals.values())
    return sum(v) / len(v), len(v)


def calibrated_traffic(kernel: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str,
                       copy_write_csv: str, copy_bytes: int) -> dict:
    f_k, nf = counter_mean(fetch_csv, kernel, "FETCH_SIZE")
    w_k, nw = counter_mean(write_csv, kernel, "WRITE_SIZE")
    f_c, _ = counter_mean(copy_fetch_csv, "copyBuffer", "FETCH_SIZE")
    w_c, _ = counter_mean(copy_write_csv, "copyBuffer", "WRITE_SIZE")
    fetch_scale = copy_bytes / (f_c * 1024.0)
    write_scale = copy_bytes / (w_c * 1024.0)
    read_b = f_k * 1024.0 * fetch_scale
    write_b = w_k * 1024.0 * write_scale
    return {"fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k, "dispatches": min(nf, nw),
            "copy_fetch_kib": f_c, "copy_write_kib": w_c, "fetch_scale": fetch_scale,
            "write_scale": write_scale, "read_bytes": read_b, "write_bytes": write_b,
            "hbm_bytes_per_launch": read_b + write_b}


def main(argv):
    if not argv:
        print(__doc__)
        return 2
    if argv[0] == "copy":
        copy_probe(float(argv[1]) if len(argv) > 1 else 1.0)
    elif argv[0] == "moments":
        a = argv[1:] + [None] * 4
        moments_probe(int(a[0] or 256), int(a[1] or 512), int(a[2] or 20), a[3] or "fp32")
    elif argv[0] == "stats":
        print(stats_markdown(argv[1]))
    elif argv[0] == "traffic":
        import json
        print(json.dumps(calibrated_traffic(argv[1], argv[2], argv[3], argv[4], argv[5], int(argv[6])), indent=1))
    elif argv[0] == "counter":
        m, n = counter_mean(argv[1], argv[2], argv[3])
        print(f"{argv[3]} mean over {n} dispatches: {m}")
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
