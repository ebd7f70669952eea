"""Helpers of the GPU parity tests: run the HIP sweep through the C-ABI and
compare with the FP64 oracle element by element."""
from __future__ import annotations

import numpy as np

# Relative tolerance on J, J_exact, Gamma (and J_in): 1e-5, with the error of a
# cell measured against max(|ref|, 1e-6 max|ref|) so that cells whose value is
# a million times below the field's maximum are judged in absolute terms.
RTOL = 1e-5
FLOOR = 1e-6


def err_stats(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), FLOOR * np.max(np.abs(ref)) if ref.size else 1.0)
    scale = np.where(scale > 0, scale, 1.0)
    e = np.abs(gpu - ref) / scale
    if e.size == 0:
        return dict(max=0.0, p999=0.0, rms=0.0)
    return dict(max=float(e.max()), p999=float(np.quantile(e, 0.999)),
                rms=float(np.sqrt(np.mean(e * e))))


def check(name, gpu, ref, rtol=RTOL, report=None):
    st = err_stats(gpu, ref)
    line = f"{name}: max {st['max']:.3e}  p99.9 {st['p999']:.3e}  rms {st['rms']:.3e}"
    print(line, flush=True)
    if report is not None:
        report[name] = st
    assert st["max"] <= rtol, line
    return st


def gpu_sweep(medium, tuning=None, I_bc=None, exit_sum=True):
    """Run art_sweep on cuda:0 and return numpy outputs."""
    import torch
    from paper_1410_0763_amd import art
    nb, nz, ny, nx = medium.kappa.shape
    with art.Mesh(nx, ny, nz, medium.cell_size) as m:
        if tuning is not None:
            m.set_tuning(**tuning) if isinstance(tuning, dict) else m.set_tuning(*tuning)
        k = torch.from_numpy(medium.kappa).cuda()
        s = torch.from_numpy(medium.S).cuda()
        m.set_fields(k, s)
        if medium.heat_in is not None:
            m.set_heating(medium.heat_in, medium.heat_src)
        out = m.sweep(medium.nside, gamma_w=medium.gamma_w,
                      I_bc=medium.I_bc if I_bc is None else I_bc, exit_sum=exit_sum)
        torch.cuda.synchronize()
        return {key: v.cpu().numpy() for key, v in out.items()}


def oracle_sweep(medium, I_bc=None, nthreads=0):
    from oracle import oracle as O
    h64 = (lambda a: None if a is None else a.astype(np.float64))
    return O.sweep(medium.kappa.astype(np.float64), medium.S.astype(np.float64), medium.nside,
                   gamma_w=medium.gamma_w.astype(np.float64), h=medium.cell_size,
                   I_bc=medium.I_bc if I_bc is None else I_bc, nthreads=nthreads,
                   heat_in=h64(medium.heat_in), heat_src=h64(medium.heat_src))


def compare_all(medium, gpu, ref, report=None, rtol=RTOL):
    for key in ("J_in", "J", "J_exact", "Gamma"):
        check(f"{medium.name}:{key}", gpu[key], ref[key], rtol=rtol, report=report)
    if medium.heat_in is not None:
        check(f"{medium.name}:Heat", gpu["Heat"], ref["Heat"], rtol=rtol, report=report)
    else:
        assert not np.any(gpu["Heat"]), "Heat must be 0 without heating weights"
    if "exit_sum" in gpu:
        # per direction and bin, relative to the largest exit sum of that bin
        g = gpu["exit_sum"].astype(np.float64)
        r = ref["exit_sum"]
        scale = np.maximum(np.abs(r).max(axis=0, keepdims=True), 1e-30)
        e = np.abs(g - r) / scale
        print(f"{medium.name}:exit_sum max {e.max():.3e}", flush=True)
        assert e.max() <= 10 * rtol
