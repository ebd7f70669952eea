"""Benchmark of the diffuse-radiation sweep on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one full sweep (direction generator, block-wavefront march,
normalisation and rates) of the 256^3 clumpy workload: lognormal density with
sigma_ln = 1.5 and 64 opaque spheres, HEALPix nside 8 (768 directions), four
frequency bins, fields resident in HBM before timing starts.  One JSON line is
printed; `value` is segment-bin updates per second (one ray-cell segment of
positive length in one frequency bin), counted by the kernels themselves.

roofline: algorithmic bytes of the march = 8 B (kappa_b and S_b read once) per
(cell, direction, bin), divided by the march phase's HIP-event time on the
sweep's stream, against the 8 TB/s HBM peak; `traffic` is the HBM byte count
of the march from the committed rocprofv3 counter summary, null when that
summary was taken on a different march kernel source.

cpu_baseline: the FP64 oracle (test infrastructure) on the host cores, on a
bounded sample of the same workload: 36 of the 768 directions (around the
equator) over the full mesh and all four bins.
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
WORKLOAD = ("plain_256: 256^3 lognormal (sigma_ln 1.5) + 64 spheres (kappa x100), "
            "HEALPix nside 8 (768 directions), 4 frequency bins, FP32")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_plain_256_traffic.json")
MARCH_SRC = os.path.join(ROOT, "paper_1410_0763_amd", "csrc", "art_march.hip")


def march_source_hash():
    with open(MARCH_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic():
    """HBM bytes per sweep of the march from the committed counter summary,
    or None when absent or taken on another march source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("march_source_sha256_16") != march_source_hash():
        return None
    return t.get("hbm_bytes_per_sweep")


COPY_BYTES = 1 << 30   # calibration copy: 1 GiB read + 1 GiB written


def copy_calibration():
    """A plain device-to-device copy of known size, run under the same
    FETCH_SIZE / WRITE_SIZE counters as the march to calibrate them."""
    import torch
    src = torch.ones(COPY_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}), flush=True)


def _pmc_sums(path, counter):
    """Per-kernel-name sums of one counter over all dispatches (KiB as
    reported), from a rocprofv3 --pmc output: its SQLite database
    (*_results.db) or its counter_collection CSV."""
    import collections
    out = collections.defaultdict(float)
    calls = collections.Counter()
    if path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(path)
        rows = con.execute("select kernel_name, value from counters_collection "
                           "where counter_name = ?", (counter,)).fetchall()
        con.close()
    else:
        import csv
        with open(path) as f:
            rows = [(r["Kernel_Name"], r["Counter_Value"]) for r in csv.DictReader(f)
                    if r["Counter_Name"] == counter]
    for name, val in rows:
        out[name] += float(val)
        calls[name] += 1
    return out, calls


def traffic_from(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, sweeps):
    """HBM bytes per sweep of the march from FETCH_SIZE and WRITE_SIZE runs,
    each scaled by what the same counter reads for the calibration copy."""
    f, fc = _pmc_sums(fetch_csv, "FETCH_SIZE")
    w, _ = _pmc_sums(write_csv, "WRITE_SIZE")
    cf, _ = _pmc_sums(copy_fetch_csv, "FETCH_SIZE")
    cw, _ = _pmc_sums(copy_write_csv, "WRITE_SIZE")
    ckey = max(cf, key=cf.get)                   # the copy kernel
    fetch_scale = COPY_BYTES / (cf[ckey] * 1024.0)
    write_scale = COPY_BYTES / (cw[ckey] * 1024.0)
    mk = [k for k in f if "art_march_kernel" in k]
    fetch = sum(f[k] for k in mk) * 1024.0 * fetch_scale / sweeps
    write = sum(w.get(k, 0.0) for k in mk) * 1024.0 * write_scale / sweeps
    rec = {"kernel": mk, "dispatches": sum(fc[k] for k in mk), "sweeps": sweeps,
           "fetch_bytes_per_sweep": fetch, "write_bytes_per_sweep": write,
           "hbm_bytes_per_sweep": fetch + write,
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "march_source_sha256_16": march_source_hash()}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


def cpu_baseline(medium, d_range=(366, 402)):
    import numpy as np
    from oracle import oracle as O
    threads = min(16, os.cpu_count() or 1)
    k = medium.kappa.astype(np.float64)
    s = medium.S.astype(np.float64)
    t0 = time.perf_counter()
    r = O.sweep_raw(k, s, medium.nside, d_range=d_range, nthreads=threads)
    dt = time.perf_counter() - t0
    units = r["nseg"] * medium.nbins
    return {"value": units / dt, "unit": "seg-bin updates/s", "cores": threads, "kind": "oracle",
            "sample": f"directions {d_range[0]}..{d_range[1] - 1} of 768, full 256^3 mesh, "
                      f"4 bins ({units:.3e} segment-bin updates in {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only the counter-calibration copy of 1 GiB")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the march traffic summary from rocprofv3 --pmc outputs "
                         "(*_results.db or counter_collection.csv)")
    ap.add_argument("--sweeps", type=int, default=1, help="sweeps in the --traffic-from runs")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, sweeps=args.sweeps)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the sweep of one mesh is measured on one MI355X; "
              "see DESIGN.md for how directions would be sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1410_0763_amd import art, media

    torch.cuda.set_device(0)
    m = media.plain_256()
    nb, nz, ny, nx = m.kappa.shape
    mesh = art.Mesh(nx, ny, nz, m.cell_size)
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
    out = mesh.alloc_outputs(m.nside)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        mesh.sweep(m.nside, gamma_w=m.gamma_w, out=out)
    torch.cuda.synchronize()

    march_ms, sweep_ms, segs = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mesh.sweep(m.nside, gamma_w=m.gamma_w, out=out)
        st = mesh.stats()          # waits for this sweep's end event
        march_ms.append(st["march_ms"])
        sweep_ms.append(st["sweep_ms"])
        segs.append(st["segments"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    seg_bins = segs[-1] * nb
    ms_per_step = 1e3 * wall / args.steps
    value = seg_bins / (sum(sweep_ms) / len(sweep_ms) / 1e3)
    nd = 12 * m.nside ** 2
    alg_bytes = 8.0 * nx * ny * nz * nd * nb
    march_s = (sum(march_ms) / len(march_ms)) / 1e3
    achieved = alg_bytes / march_s / 1e9
    traffic = load_traffic()
    # the march is one launch per wavefront index: the largest block-index sum
    # over the three dominant axes, plus one
    tn = mesh.get_tuning()
    dims = (nx, ny, nz)
    launches = max(-(-dims[a] // tn["depth"]) + sum(-(-dims[q] // 8) for q in range(3) if q != a) - 2
                   for a in range(3))
    rec = {
        "metric": "ray-segment updates/s (segment-bin updates per second) of the plain FP32 sweep",
        "value": value,
        "unit": "seg-bin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "mesh": [nx, ny, nz], "nside": m.nside, "nbins": nb,
                   "directions": nd, "tuning": mesh.get_tuning(),
                   "segments_per_bin": segs[-1], "sweep_ms_event": sum(sweep_ms) / len(sweep_ms),
                   "march_ms_event": sum(march_ms) / len(march_ms)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / launches,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "algorithmic_bytes_per_launch": alg_bytes / launches,
                     "algorithmic_bytes_per_sweep": alg_bytes,
                     "launches_per_sweep": launches,
                     "avg_launch_ms": 1e3 * march_s / launches,
                     "kernel": f"art_march_kernel<{nb},{tn['interleave']}> "
                               "(achieved = algorithmic bytes per launch / average launch time)"},
        "cpu_baseline": None,
    }
    mesh.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(m)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
