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
equator) over the full mesh and all four bins on every core of the process's
CPU share (at most 16), and 2 directions on one core (`value_1core`); `nproc`
and the CPU share are reported with it.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = ("plain_256: 256^3 lognormal (sigma_ln 1.5) + 64 spheres (kappa x100), "
            "HEALPix nside 8 (768 directions), 4 frequency bins, FP32")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_plain_256_traffic.json")
MARCH_SRC = os.path.join(ROOT, "paper_1410_0763_amd", "csrc", "art_march.hip")


def copy_rate_gbs(nbytes=2 << 30, reps=5):
    """HBM rate a plain device-to-device copy of nbytes reaches on this GPU
    (bytes read + written per second, in GB/s), measured after the timed
    region: what streaming code attains here, beside the published peak."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms / 1e3) / 1e9


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


POINT_SRC = os.path.join(ROOT, "paper_1410_0763_amd", "csrc", "art_point.hip")
POINT_VALU_FILE = os.path.join(ROOT, "profiles", "point_128_valu.json")
# vector-ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave
# instruction occupies a SIMD for 4 cycles; FP64 and FP32 alike)
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X, FP64 vector (an FMA counts 2)


def point_valu_per_segment():
    """Vector-ALU lane-instructions per segment of the point-source kernel from
    the committed counter summary, or None when absent or taken on another
    kernel source."""
    try:
        with open(POINT_VALU_FILE) as f:
            t = json.load(f)
        with open(POINT_SRC, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if t.get("point_source_sha256_16") != h:
        return None
    return t.get("valu_lane_instructions_per_segment")


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


def cpu_baseline(medium, d_range=(366, 402), d_range_1=(366, 368)):
    """The FP64 oracle on this host's cores: on every core of the process's
    CPU share (at most 16, the share of one GPU) over 36 directions, and on
    one core over 2 of them; the rate is work-additive over directions."""
    import numpy as np
    from oracle import oracle as O
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(16, share))
    k = medium.kappa.astype(np.float64)
    s = medium.S.astype(np.float64)

    def run(rng, nthreads):
        t0 = time.perf_counter()
        r = O.sweep_raw(k, s, medium.nside, d_range=rng, nthreads=nthreads)
        dt = time.perf_counter() - t0
        return r["nseg"] * medium.nbins, dt

    units, dt = run(d_range, threads)
    units1, dt1 = run(d_range_1, 1)
    return {"value": units / dt, "unit": "seg-bin updates/s", "cores": threads, "kind": "oracle",
            "sample": f"directions {d_range[0]}..{d_range[1] - 1} of 768, full 256^3 mesh, "
                      f"4 bins ({units:.3e} segment-bin updates in {dt:.1f} s on {threads} threads)",
            "nproc": os.cpu_count(), "cpu_share": share,
            "value_1core": units1 / dt1,
            "sample_1core": f"directions {d_range_1[0]}..{d_range_1[1] - 1}, full mesh, 4 bins "
                            f"({units1:.3e} segment-bin updates in {dt1:.1f} s on 1 thread)"}


BATCH_CANDIDATES = [dict(depth=d, subsets=1, waves=1, interleave=k)
                    for d in (3, 4, 6, 8) for k in (2, 3, 4)]
# depth only, every mesh keeping 3 directions per wave: the batch's launches
# then group by bin count alone (at most four chains, one per hardware queue)
BATCH_DEPTH_CANDIDATES = [dict(depth=d, subsets=1, waves=1, interleave=3) for d in (3, 4, 5, 6, 8)]


def bench_batched(count=48, reps=5):
    """The uneven batch (48 meshes, sides 32-128, Nside 2/4/8, 1-4 bins): one
    graph replay of the batched form against the 48 plain sweeps it replaces,
    each timed the same way (HIP events around the whole, best of `reps`
    after one warm-up), first with every mesh at the default launch shape,
    then with each mesh autotuned through the library's shape-class cache."""
    import torch
    from paper_1410_0763_amd import art, media
    meds = media.batch_media(count=count)
    meshes = []
    for m in meds:
        nb, nz, ny, nx = m.kappa.shape
        mesh = art.Mesh(nx, ny, nz, m.cell_size)
        mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
        meshes.append(mesh)
    outs = [mesh.alloc_outputs(m.nside) for mesh, m in zip(meshes, meds)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best_of(fn):
        fn()                                   # warm-up (allocations, tables)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def plain():
        for mesh, m, o in zip(meshes, meds, outs):
            mesh.sweep(m.nside, gamma_w=m.gamma_w, out=o)

    def measure(tag):
        plain_ms = best_of(plain)
        batch = art.Batch(meshes, [m.nside for m in meds], [m.gamma_w for m in meds])
        batch_ms = best_of(lambda: batch.launch())
        st = batch.stats()
        batch.close()
        return dict(batch_ms=batch_ms, plain_48_calls_ms=plain_ms, segment_bins=st["segment_bins"],
                    value=st["segment_bins"] / (batch_ms / 1e3),
                    plain_value=st["segment_bins"] / (plain_ms / 1e3),
                    speedup_vs_plain=plain_ms / batch_ms)

    default = measure("default")

    def tune(cands):
        art.tune_cache("clear")
        t0 = time.perf_counter()
        tunings, cached = [], 0
        for mesh, m in zip(meshes, meds):
            r = mesh.autotune_class(m.nside, candidates=cands)
            tunings.append(r["tuning"])
            cached += int(r["cached"])
        info = {"seconds": time.perf_counter() - t0, "meshes": count, "cache_hits": cached,
                "classes": count - cached, "candidates": len(cands),
                "shapes_chosen": sorted({(t["depth"], t["interleave"]) for t in tunings})}
        return measure("tuned"), info

    tuned, tune_info = tune(BATCH_CANDIDATES)
    tuned_d, tune_d_info = tune(BATCH_DEPTH_CANDIDATES)
    variants = {"default": default, "autotuned": tuned, "autotuned_depth": tuned_d}
    kept = min(variants, key=lambda k: variants[k]["batch_ms"])
    best = variants[kept]
    rec = {"metric": "segment-bin updates/s of the batched form (48 uneven meshes, one graph replay)",
           "value": best["value"], "unit": "seg-bin updates/s",
           "batch_ms": best["batch_ms"], "plain_48_calls_ms": best["plain_48_calls_ms"],
           "speedup_vs_plain": best["speedup_vs_plain"], "segment_bins": best["segment_bins"],
           "kept": kept, "default": default, "autotuned": tuned, "autotuned_depth": tuned_d,
           "autotune": tune_info, "autotune_depth": tune_d_info,
           "timing": f"HIP events around the whole replay / the 48 calls, best of {reps} after a warm-up",
           "config": {"workload": "48 meshes, sides 32-128 (a third cubes), lognormal sigma_ln 1, "
                                  "Nside 2/4/8, 1-4 bins, seeds 4000+i"}}
    for mesh in meshes:
        mesh.close()
    print(json.dumps(rec), flush=True)


def bench_surrogate(train_fields=512, steps=9600, lam=1.0, test_fields=64):
    """128^3, Nside 2 -> 16: time of coarse sweep + network inference against
    the fine sweep, held-out errors (the gate's relative L2 of J and the
    per-cell log error), and the conv layer's matrix-core rate.  Inputs are
    the coarse sweep's J, the log density and the neutral fraction."""
    import torch
    from paper_1410_0763_amd import art, media
    from paper_1410_0763_amd import surrogate as SG
    from paper_1410_0763_amd.art import nn
    shape = (128, 128, 128)
    V = 128 ** 3
    model = SG.Surrogate(shape, seed=0)
    mesh = art.Mesh(*shape)

    def pairs(idx, train):
        out = []
        for i in idx:
            m = media.surrogate_medium(i, train=train)
            k, s = torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda()
            mesh.set_fields(k, s)
            t = torch.zeros(V, dtype=torch.float32, device="cuda")
            w = torch.zeros(V, dtype=torch.float32, device="cuda")
            Jc, Jf = SG.make_pair(mesh, model, 2, 16, t, w, lam=lam)
            out.append(dict(k=k, s=s, t=t, w=w, Jc=Jc, Jf=Jf,
                            n=torch.from_numpy(m.density).cuda().reshape(-1),
                            xh=torch.from_numpy(m.x_hi).cuda().reshape(-1)))
        return out
    t0 = time.perf_counter()
    train = pairs(range(train_fields), True)
    model.fit_stats([p["Jc"] for p in train[:4]], [p["n"] for p in train[:4]],
                    [p["xh"] for p in train[:4]], margin=1.0)
    for p in train:
        p["x"] = torch.zeros((V, 16), dtype=torch.int16, device="cuda")
        model.features(p["Jc"], p["n"], p["xh"], p["x"])
    test = pairs(range(test_fields), False)
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    for it in range(steps):
        lr = 1e-3 * 0.5 * (1 + np.cos(np.pi * it / steps)) + 1e-5
        p = train[it % len(train)]
        model.train_step(p["x"], p["t"], lr=lr, weight=p["w"])
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    lr_c, lr_s, l2_c, l2_s = [], [], [], []
    model.set_val_err(0.0)
    for p in test:
        mesh.set_fields(p["k"], p["s"])
        out, fb, _ = SG.sweep_surrogate(mesh, model, p["n"], p["xh"], 2, 16, err_bound=1e9)
        J = out["J"].reshape(-1)
        Jf = p["Jf"]
        lr_s.append(torch.sqrt(torch.mean(torch.log(J / Jf) ** 2)).item())
        lr_c.append(torch.sqrt(torch.mean(torch.log(p["Jc"] / Jf) ** 2)).item())
        l2_s.append((torch.linalg.norm(J - Jf) / torch.linalg.norm(Jf)).item())
        l2_c.append((torch.linalg.norm(p["Jc"] - Jf) / torch.linalg.norm(Jf)).item())
    model.set_val_err(float(np.mean(l2_s)))
    p = test[0]
    mesh.set_fields(p["k"], p["s"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best
    sout = mesh.alloc_outputs(16)
    used = []

    def sur():
        _, fb, _ = SG.sweep_surrogate(mesh, model, p["n"], p["xh"], 2, 16, err_bound=1.0, out=sout)
        used.append(fb)
    sur_ms = timed(sur)
    assert not any(used), "the gate fell back during the timed surrogate calls"
    fine_ms = timed(lambda: mesh.sweep(16))
    coarse_ms = timed(lambda: mesh.sweep(2))
    x = torch.zeros((V, 16), dtype=torch.int16, device="cuda")
    model.features(p["Jc"], p["n"], p["xh"], x)
    infer_ms = timed(lambda: model.forward(x))
    # one 32 -> 32 channel layer (the network's dominant kernel) on the trained
    # layer-1 weights and the layer-0 activations of a held-out field
    wk = [(torch.zeros((27, 32, c), dtype=torch.int16, device="cuda"),
           torch.zeros((27, 32, 32), dtype=torch.int16, device="cuda")) for c in (16, 32)]
    for l, (wf, wb) in enumerate(wk):
        nn.prep_weights(model.param(l, SG.W), SG.CIN[l], wf, wb)
    xa = torch.zeros((V, 32), dtype=torch.int16, device="cuda")
    y = torch.zeros((V, 32), dtype=torch.int16, device="cuda")
    b0, b1 = model.param(0, SG.B), model.param(1, SG.B)
    nn.conv3d_fwd(x, 16, wk[0][0], b0, shape, 1, y=xa)
    wf = wk[1][0]
    conv_ms = timed(lambda: nn.conv3d_fwd(xa, 32, wf, b1, shape, 1, y=y), 20)
    conv_flop = 2.0 * 27 * 32 * 32 * V
    # weight and bias gradients of the same layer (its input xa, the layer
    # output y standing in for the gradient), workspace partials summed
    work = torch.zeros(nn.bwd_weight_workspace(32, shape), dtype=torch.float32, device="cuda")
    dw = torch.zeros((27, 32, 32), dtype=torch.float32, device="cuda")
    db = torch.zeros(32, dtype=torch.float32, device="cuda")
    bwdw_ms = timed(lambda: nn.conv3d_bwd_weight(xa, 32, y, shape, work, dw, db), 20)
    rec = {"metric": "surrogate: coarse sweep + inference time against the fine sweep (128^3, Nside 2 -> 16)",
           "value": fine_ms / sur_ms, "unit": "x faster than the fine sweep",
           "surrogate_ms": sur_ms, "fine_sweep_ms": fine_ms, "coarse_sweep_ms": coarse_ms,
           "inference_ms": infer_ms, "train_steps": steps, "train_s": train_s, "loss_lambda": lam,
           "train_fields": train_fields, "held_out_fields": test_fields, "data_s": data_s,
           "inputs": "log J (Nside 2), log n, x_HI; target log(J_in at Nside 16 / J_in at Nside 2)",
           "held_out_log_rms": {"coarse": float(np.mean(lr_c)), "surrogate": float(np.mean(lr_s))},
           "held_out_rel_l2": {"coarse": float(np.mean(l2_c)), "surrogate": float(np.mean(l2_s))},
           "params": model.n_params(),
           "roofline": {"bound": "mfma", "kernel": "conv3d_fwd_kernel<32> (one 32->32 layer, 128^3)",
                        "achieved": conv_flop / (conv_ms / 1e3) / 1e12, "peak": 2500.0,
                        "unit": "TFLOP/s", "frac": conv_flop / (conv_ms / 1e3) / 1e12 / 2500.0,
                        "layer_ms": conv_ms},
           "weight_gradient": {"kernel": "conv3d_bwd_weight (32->32 layer, 128^3, with the bias and the "
                                         "partial sums)", "ms": bwdw_ms,
                               "tflops": conv_flop / (bwdw_ms / 1e3) / 1e12,
                               "frac": conv_flop / (bwdw_ms / 1e3) / 1e12 / 2500.0},
           "train_step_ms": train_s / steps * 1e3,
           "config": {"workload": f"128^3 lognormal sigma_ln 1.5 + 16 spheres, 1 bin; {train_fields} "
                                  f"training fields (seeds 5000+i), {test_fields} held-out (6000+i)"}}
    mesh.close()
    print(json.dumps(rec), flush=True)


def bench_point(steps=5, cpu=True):
    """Point-source rates (Sect. 2.3, Appendix A) on the 128^3 clumpy medium
    with 16 sources and 4 bins: HIP events around art_point_sources; the
    oracle timed on a bounded sample of target cells beside it."""
    import numpy as np
    import torch
    from paper_1410_0763_amd import art, media
    w = media.point_sources()
    m = w.medium
    nb, nz, ny, nx = m.kappa.shape
    mesh = art.Mesh(nx, ny, nz, m.cell_size)
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
    nab = torch.from_numpy(w.n_abs).cuda()
    out = mesh.point_sources(w.pos, w.Q, nab, e=w.e, segs=True)
    torch.cuda.synchronize()
    segs = int(out["segs"].to(torch.int64).sum().item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        mesh.point_sources(w.pos, w.Q, nab, e=w.e, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rec = {"metric": "segment-bin updates/s of point-source RT (photon-conserving rates)",
           "value": segs * nb / (ms / 1e3), "unit": "seg-bin updates/s", "n_gpus": 1,
           "steps": steps, "ms_per_step": ms, "higher_is_better": True, "dtype": "f64 geometry, f32 fields",
           "data": "synthetic", "segments": segs,
           "config": {"workload": "128^3 lognormal (sigma_ln 1.5) + 16 opaque spheres, 16 point "
                                  "sources, 4 bins", "kernel": "art_point_kernel<4>"}}
    # the method's FP64 work per walk segment (Sect. 2.3): the nearest of the
    # three next plane crossings (2 comparisons), the segment length (1), the
    # next crossing of the axis crossed (1), and tau_b += kappa_b h dl per bin
    # (one fused multiply-add = 2 flops each); against the FP64 vector peak
    flops_per_seg = 4 + 2 * nb
    achieved = flops_per_seg * segs / (ms / 1e3) / 1e12
    rec["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                       "flops_per_segment": flops_per_seg, "traffic": None}
    vps = point_valu_per_segment()
    if vps is not None:           # measured issue, for reference (not the roofline)
        rec["valu_lane_instructions_per_segment"] = vps
        rec["valu_issue_frac"] = vps * segs / (ms / 1e3) / VALU_LANE_PEAK
    if cpu:
        from oracle import oracle as O
        threads = min(16, os.cpu_count() or 1)
        t0 = time.perf_counter()
        O.point(m.kappa, w.n_abs, w.pos, w.Q, w.e, nthreads=threads)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": segs * nb / dt, "unit": "seg-bin updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"the whole workload ({nx * ny * nz} target cells x "
                                         f"{len(w.pos)} sources x {nb} bins) in {dt:.1f} s"}
    mesh.close()
    print(json.dumps(rec), flush=True)


def bench_chem(steps=5, cpu=True):
    """Chemistry and energy update (Appendices B-D) of every cell of a 128^3
    medium, driven by the rates of its own Nside 2 sweep: HIP events around
    art_chem_step, the FP64 oracle timed on a sample of cells beside it."""
    import numpy as np
    import torch
    from paper_1410_0763_amd import art, media
    m = media.clumpy_medium((128, 128, 128), nside=2, sigma_ln=1.5, seed=5100, spheres=16, name="chem128")
    nb, nz, ny, nx = m.kappa.shape
    n = nx * ny * nz
    mesh = art.Mesh(nx, ny, nz)
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
    mesh.set_heating([1.5], [0.1])
    out = mesh.sweep(m.nside)
    G = out["Gamma"].reshape(-1).contiguous()
    H = out["Heat"].reshape(-1).contiguous()
    lt = np.linspace(1.0, 9.0, 81)
    T = 10.0 ** lt
    tabs = dict(alpha=2.0 * (T / 1e4) ** -0.7, k_ci=0.5 * np.exp(-1.6e5 / T),
                cool_I=3e-2 * np.exp(-1.2e5 / T), cool_II=1e-4 * (T / 1e4) ** 0.5)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    tables = {k: d(v) for k, v in tabs.items()}
    nH = d(m.density.reshape(-1))
    x0, u0 = m.x_hi.reshape(-1).astype(np.float64), np.full(n, 300.0)
    xg, ug = d(x0), d(u0)
    ns = torch.empty(n, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(steps + 1):
        xg.copy_(d(x0))
        ug.copy_(d(u0))
        torch.cuda.synchronize()
        e0.record()
        art.chem_step(nH, nH, G, H, xg, ug, 0.5, tables, 1.0, 0.1, T_per_u=10.0, nsub=ns)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = min(times[1:])
    subs = int(ns.to(torch.int64).sum().item())
    rec = {"metric": "cells/s of the chemistry and energy update (Appendices B-D, hydrogen network)",
           "value": n / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": steps, "ms_per_step": ms,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "substeps": subs, "substep_cells_per_s": subs / (ms / 1e3),
           "config": {"workload": "128^3 lognormal (sigma_ln 1.5) + 16 spheres, rates of its Nside 2 "
                                  "sweep, one radiative step dt = 0.5, 81-point synthetic rate tables"},
           "roofline": None}
    if cpu:
        from oracle import chem as C
        p = C.default_params(nT=81, logT_min=1.0, logT_max=9.0, **tabs)
        p.update(T_per_u=10.0)
        idx = np.random.default_rng(1).integers(0, n, 400)
        Gc = G.cpu().numpy().astype(np.float64)
        Hc = H.cpu().numpy().astype(np.float64)
        nHc = m.density.reshape(-1).astype(np.float64)
        t0 = time.perf_counter()
        C.step(nHc[idx], nHc[idx], Gc[idx], Hc[idx], x0[idx], u0[idx], 0.5, p)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": len(idx) / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
                               "sample": f"{len(idx)} random cells of the same step in {dt:.1f} s "
                                         "(plain Python loops)"}
    mesh.close()
    print(json.dumps(rec), flush=True)


def bench_rtchem(steps=3, cpu=True):
    """One radiative step coupled to the chemistry (Appendix D iteration) on a
    128^3 medium, Nside 2, one bin: wall time of art_rt_chem_step (it waits
    for the stream after every iteration), its iteration count; the FP64
    oracle timed on a small mesh beside it."""
    import numpy as np
    import torch
    from paper_1410_0763_amd import art, media
    m = media.clumpy_medium((128, 128, 128), nside=2, sigma_ln=1.5, seed=5100, spheres=16, name="rtchem128")
    _, nz, ny, nx = m.kappa.shape
    n = nx * ny * nz
    lt = np.linspace(1.0, 9.0, 81)
    T = 10.0 ** lt
    alpha = 2.0 * (T / 1e4) ** -0.7
    tabs = dict(alpha=alpha, k_ci=0.5 * np.exp(-1.6e5 / T), cool_I=3e-2 * np.exp(-1.2e5 / T),
                cool_II=1e-4 * (T / 1e4) ** 0.5)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    tables = {k: d(v) for k, v in tabs.items()}
    dal = d(0.38 * alpha)
    nH = d(m.density.reshape(-1))
    rho = nH * 1.2
    x0, u0 = m.x_hi.reshape(-1).astype(np.float64), np.full(n, 300.0)
    xg, ug = d(x0), d(u0)
    mesh = art.Mesh(nx, ny, nz)
    mesh_ws = art.load().art_rt_chem_workspace(mesh._h, 1)
    work = torch.empty(mesh_ws, dtype=torch.uint8, device="cuda")
    # 16 point sources, uniform in the box, photon rates log-uniform over two decades
    srng = np.random.default_rng(5150)
    spos = srng.uniform(0.0, 1.0, size=(16, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    sQ = 1e4 * 10.0 ** srng.uniform(-1.0, 1.0, size=(16, 1))
    kw = dict(nside=2, gamma_w=[1.0], heat_in=[3.0], heat_src=[1.0], T_per_u=10.0, max_iter=100, work=work,
              sources=(spos, sQ, [0.5]))
    times, its = [], []
    for _ in range(steps + 1):
        xg.copy_(d(x0))
        ug.copy_(d(u0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = art.rt_chem_step(mesh, nH, rho, xg, ug, 0.3, tables, 1.0, 0.1, [2.0], [1.0], dal, **kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        its.append(r["iterations"])
    ms = min(times[1:])
    it = its[-1]
    rec = {"metric": "cell-iterations/s of the radiative step coupled to the chemistry (Appendix D)",
           "value": n * it / (ms / 1e3), "unit": "cell-iterations/s", "n_gpus": 1, "steps": steps,
           "ms_per_step": ms, "iterations": it, "converged": r["converged"],
           "ms_per_iteration": ms / it, "dt_chem_min": r["dt_chem_min"], "workspace_bytes": int(mesh_ws),
           "higher_is_better": True, "dtype": "f64 (chemistry), f32 (sweep)", "data": "synthetic",
           "config": {"workload": "128^3 lognormal (sigma_ln 1.5) + 16 spheres as n_H, its x_HI; Nside 2, "
                                  "1 bin, sigma 2, dalpha = 0.38 alpha, 16 point sources (Q 1e3-1e5, e 0.5), "
                                  "dt = 0.3, 81-point synthetic tables"},
           "roofline": None}
    # the same interval in radiative steps of F = 4 minimum chemical timesteps
    # (art_rt_chem_advance, time stepping of Appendix D)
    xg.copy_(d(x0))
    ug.copy_(d(u0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a = art.rt_chem_advance(mesh, nH, rho, xg, ug, 0.3, 4.0, tables, 1.0, 0.1, [2.0], [1.0], dal, **kw)
    torch.cuda.synchronize()
    ams = (time.perf_counter() - t0) * 1e3
    rec["advance"] = {"t_end": 0.3, "F": 4.0, "steps": a["steps"], "iterations": a["iterations"],
                      "unconverged": a["unconverged"], "t": a["t"], "ms": ams,
                      "cell_iterations_per_s": n * (a["iterations"] + 1) / (ams / 1e3),
                      "note": "iterations over the radiative steps plus the length-0 step that gives the "
                              "first chemical timestep"}
    if cpu:
        from oracle import chem as C
        from oracle import rtchem as RC
        cp = C.default_params(nT=81, logT_min=1.0, logT_max=9.0, **tabs)
        cp.update(T_per_u=10.0)
        rp = RC.default_rt_params(nT=81, dalpha=0.38 * alpha, sigma=[2.0], heat_in=[3.0], heat_src=[1.0],
                                  nside=2, src_pos=[[2.0, 3.0, 4.0], [6.0, 1.0, 1.5]], src_Q=[[1e3], [1e4]],
                                  src_e=[0.5])
        shp = (6, 8, 8)
        sn = int(np.prod(shp))
        rng = np.random.default_rng(2)
        sH = rng.lognormal(0.0, 0.7, sn)
        t0 = time.perf_counter()
        ref = RC.step(shp, 1.0, sH, sH * 1.2, rng.uniform(0.05, 0.95, sn), np.full(sn, 300.0), 0.3, rp, cp, 100)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": sn * ref["iterations"] / dt, "unit": "cell-iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"a {shp} mesh of the same recipe with 2 sources, {ref['iterations']} "
                                         f"iterations in {dt:.1f} s (FP64 sweep and point rates in C, "
                                         "chemistry in Python loops)"}
    mesh.close()
    print(json.dumps(rec), flush=True)


def bench_bwd_weight(reps=20):
    """Weight and bias gradients of one 32 -> 32 and one 16 -> 32 layer at
    128^3 (random bf16 operands): HIP events around art_conv3d_bwd_weight
    (products and the fixed-order partial sums), best of 5 runs of reps calls."""
    import numpy as np
    import torch
    from paper_1410_0763_amd.art import nn
    shape = (128, 128, 128)
    V = 128 ** 3
    rng = np.random.default_rng(1)
    g = torch.from_numpy(rng.integers(-20000, 20000, size=(V, 32), dtype=np.int16)).cuda()
    x32 = torch.from_numpy(rng.integers(-20000, 20000, size=(V, 32), dtype=np.int16)).cuda()
    rows = []
    for cin in (32, 16):
        x = x32[:, :cin].contiguous()
        work = torch.zeros(nn.bwd_weight_workspace(cin, shape), dtype=torch.float32, device="cuda")
        dw = torch.zeros((27, cin, 32), dtype=torch.float32, device="cuda")
        db = torch.zeros(32, dtype=torch.float32, device="cuda")
        for _ in range(3):
            nn.conv3d_bwd_weight(x, cin, g, shape, work, dw, db)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = 1e30
        for _ in range(5):
            e0.record()
            for _ in range(reps):
                nn.conv3d_bwd_weight(x, cin, g, shape, work, dw, db)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / reps)
        flop = 2.0 * 27 * 32 * 32 * V          # the 16-channel layer fills half of each tile
        rows.append({"cin": cin, "ms": best, "tflops_of_32x32_work": flop / (best / 1e3) / 1e12,
                     "frac": flop / (best / 1e3) / 1e12 / 2500.0})
    print(json.dumps({"metric": "ms per weight+bias gradient of a conv3d layer (128^3, 27 taps, 32 out "
                                "channels)", "rows": rows, "peak_tflops": 2500.0}), flush=True)


def bench_conv_fwd(reps=20):
    """Forward convolution of one 32 -> 32 and one 16 -> 32 layer at 128^3
    (random bf16 input and weights, bias, ReLU): HIP events around
    art_conv3d_fwd, best of 5 runs of reps calls."""
    import numpy as np
    import torch
    from paper_1410_0763_amd.art import nn
    shape = (128, 128, 128)
    V = 128 ** 3
    rng = np.random.default_rng(2)
    x32 = torch.from_numpy(rng.integers(-20000, 20000, size=(V, 32), dtype=np.int16)).cuda()
    y = torch.zeros((V, 32), dtype=torch.int16, device="cuda")
    bias = torch.zeros(32, dtype=torch.float32, device="cuda")
    rows = []
    for cin in (32, 16):
        x = x32[:, :cin].contiguous()
        w = torch.from_numpy((rng.normal(size=(27, cin, 32)) * 0.05).astype(np.float32)).cuda()
        wf = torch.zeros((27, 32, cin), dtype=torch.int16, device="cuda")
        wb = torch.zeros((27, 32, 32), dtype=torch.int16, device="cuda")
        nn.prep_weights(w, cin, wf, wb)
        for _ in range(3):
            nn.conv3d_fwd(x, cin, wf, bias, shape, 1, y=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = 1e30
        for _ in range(5):
            e0.record()
            for _ in range(reps):
                nn.conv3d_fwd(x, cin, wf, bias, shape, 1, y=y)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / reps)
        flop = 2.0 * 27 * cin * 32 * V
        rows.append({"cin": cin, "ms": best, "tflops": flop / (best / 1e3) / 1e12,
                     "frac": flop / (best / 1e3) / 1e12 / 2500.0})
    print(json.dumps({"metric": "ms per forward conv3d layer (128^3, 27 taps, 32 out channels, bias, ReLU)",
                      "rows": rows, "peak_tflops": 2500.0}), flush=True)


class Phases:
    """roctx ranges around the benchmark's phases (setup, warm-up, timed
    sweeps, CPU baseline), visible with rocprofv3 --marker-trace; a no-op
    where the roctx library is absent."""

    def __init__(self):
        self._lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so"):
            try:
                self._lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self._lib is not None:
            self._lib.roctxRangePushA.argtypes = [ctypes.c_char_p]

    def push(self, name):
        if self._lib is not None:
            self._lib.roctxRangePushA(name.encode())

    def pop(self):
        if self._lib is not None:
            self._lib.roctxRangePop()


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
    ap.add_argument("--batched", action="store_true",
                    help="measure the batched form (48 meshes) instead of the 256^3 sweep")
    ap.add_argument("--surrogate", action="store_true",
                    help="measure the learned surrogate (128^3) instead of the 256^3 sweep")
    ap.add_argument("--point", action="store_true",
                    help="measure point-source RT (128^3, 16 sources) instead of the 256^3 sweep")
    ap.add_argument("--sg-fields", type=int, default=512, help="training fields of --surrogate")
    ap.add_argument("--sg-steps", type=int, default=9600, help="training steps of --surrogate")
    ap.add_argument("--sg-test", type=int, default=64, help="held-out fields of --surrogate")
    ap.add_argument("--release-cost", action="store_true",
                    help="measure the cost of agent-scope release/acquire per workgroup")
    ap.add_argument("--chem", action="store_true",
                    help="measure the chemistry and energy update (128^3) instead of the 256^3 sweep")
    ap.add_argument("--conv-fwd", action="store_true",
                    help="time the surrogate's forward convolution on one 128^3 layer")
    ap.add_argument("--bwd-weight", action="store_true",
                    help="time the surrogate's weight-gradient kernel on one 128^3 layer")
    ap.add_argument("--rtchem", action="store_true",
                    help="measure a radiative step coupled to the chemistry (128^3, Nside 2)")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, sweeps=args.sweeps)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the sweep of one mesh is measured on one MI355X. "
              "Across GPUs each would sweep a contiguous range of the directions "
              "(art_sweep_range, ranges balanced by segment count) and one all-reduce of the "
              "per-cell sums would precede the normalisation; that path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1410_0763_amd import art, media

    torch.cuda.set_device(0)
    if args.batched:
        bench_batched()
        return
    if args.surrogate:
        bench_surrogate(train_fields=args.sg_fields, steps=args.sg_steps, test_fields=args.sg_test)
        return
    if args.point:
        bench_point(steps=args.steps, cpu=not args.no_cpu_baseline)
        return
    if args.release_cost:
        rows = [dict(words=w, **art.release_cost(40000, w)) for w in (256, 1024, 4096)]
        print(json.dumps({"metric": "ns per workgroup (40000 one-wave workgroups, best of 5)",
                          "rows": rows}), flush=True)
        return
    if args.chem:
        bench_chem(steps=args.steps, cpu=not args.no_cpu_baseline)
        return
    if args.rtchem:
        bench_rtchem(steps=args.steps, cpu=not args.no_cpu_baseline)
        return
    if args.bwd_weight:
        bench_bwd_weight()
        return
    if args.conv_fwd:
        bench_conv_fwd()
        return
    ph = Phases()
    ph.push("setup: medium, mesh, fields")
    m = media.plain_256()
    nb, nz, ny, nx = m.kappa.shape
    mesh = art.Mesh(nx, ny, nz, m.cell_size)
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
    out = mesh.alloc_outputs(m.nside)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ph.pop()

    ph.push("warm-up sweeps")
    for _ in range(args.warmup):
        mesh.sweep(m.nside, gamma_w=m.gamma_w, out=out)
    torch.cuda.synchronize()
    ph.pop()

    march_ms, sweep_ms, segs = [], [], []
    torch.cuda.synchronize()
    ph.push("timed sweeps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mesh.sweep(m.nside, gamma_w=m.gamma_w, out=out)
        st = mesh.stats()          # waits for this sweep's end event
        march_ms.append(st["march_ms"])
        sweep_ms.append(st["sweep_ms"])
        segs.append(st["segments"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph.pop()

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
    # the plain-VALU ceiling beside the HBM one: per segment-bin the method's
    # arithmetic is about 10 FP32 operations and one exponential (a quarter
    # of the rate: 4 issue slots), against 1024 SIMDs x 16 lanes x 2.4 GHz of
    # FP32 issue without packed math
    slots = 14
    valu_floor_ms = 1e3 * seg_bins * slots / VALU_LANE_PEAK
    rec["valu_ceiling"] = {"slots_per_segment_bin": slots, "lane_slots_per_s": VALU_LANE_PEAK,
                           "floor_ms": valu_floor_ms, "march_ms": 1e3 * march_s,
                           "frac": valu_floor_ms / (1e3 * march_s)}
    rec["config"]["sweep_ms_median"] = float(sorted(sweep_ms)[len(sweep_ms) // 2])
    mesh.close()
    ph.push("device copy reference")
    copy = copy_rate_gbs()
    rec["roofline"]["copy_GBps"] = copy
    rec["roofline"]["frac_of_copy"] = achieved / copy
    ph.pop()
    if not args.no_cpu_baseline:
        ph.push("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(m)
        ph.pop()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
