"""Independent brute-force geometry and transfer for tiny meshes.

Written from the definitions only, sharing no code with the oracle: the ray
lattice is re-stated from the reading used throughout (rays at half-integer
lattice points of the upstream face of the dominant axis, unit spacing), each
(ray, cell) chord is found by clipping the line against that one cell's box
(slab method), and intensities come from numerically integrating
dI/dl = kappa (S - I) with RK4 sub-steps and averaging them with quadrature.
"""
from __future__ import annotations

import numpy as np

TIE = 1e-12


def dominant(n):
    """Dominant axis (lowest index among components within 1e-12 of the max),
    the two others in increasing order, sign, |n_a| and the slopes."""
    m = np.max(np.abs(n))
    a = int(np.nonzero(np.abs(n) >= m - TIE)[0][0])
    b, c = [ax for ax in range(3) if ax != a]
    w = abs(n[a])
    return a, b, c, (1 if n[a] > 0 else -1), w, n[b] / w, n[c] / w


def line(n, shape_xyz, j, k):
    """Ray (j,k) as origin p0 (depth 0) and derivative dp/ds in world axes."""
    a, b, c, sig, w, tb, tc = dominant(n)
    p0 = np.zeros(3)
    v = np.zeros(3)
    p0[a] = 0.0 if sig > 0 else shape_xyz[a]
    v[a] = float(sig)
    p0[b], v[b] = j + 0.5, tb
    p0[c], v[c] = k + 0.5, tc
    return p0, v, w


def clip_box(p0, v, lo, hi):
    """Depth interval of the line p0 + v s inside the box [lo, hi] (slab method)."""
    s_lo, s_hi = -np.inf, np.inf
    for ax in range(3):
        if v[ax] == 0.0:
            if not (lo[ax] < p0[ax] < hi[ax]):
                return None
            continue
        t0 = (lo[ax] - p0[ax]) / v[ax]
        t1 = (hi[ax] - p0[ax]) / v[ax]
        s_lo = max(s_lo, min(t0, t1))
        s_hi = min(s_hi, max(t0, t1))
    if s_hi > s_lo:
        return s_lo, s_hi
    return None


def ray_chords(n, shape_zyx, j, k, h=1.0):
    """All (cell, s_in, s_out) of ray (j,k), by clipping every cell; sorted by s_in.
    Chords shorter than 1e-12 (edge/corner contacts) are dropped."""
    nz, ny, nx = shape_zyx
    N = np.array([nx, ny, nz], dtype=float)
    p0, v, w = line(n, N, j, k)
    box = clip_box(p0, v, np.zeros(3), N)
    if box is None:
        return [], w
    out = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                r = clip_box(p0, v, np.array([x, y, z], float), np.array([x + 1, y + 1, z + 1], float))
                if r is not None and r[1] - r[0] > 1e-12:
                    out.append(((z * ny + y) * nx + x, r[0], r[1]))
    out.sort(key=lambda t: t[1])
    return out, w


def lattice_rays(n, shape_zyx):
    """Every (j,k) with a positive chord, found by scanning a generous range."""
    nz, ny, nx = shape_zyx
    N = np.array([nx, ny, nz], dtype=float)
    a, b, c, sig, w, tb, tc = dominant(n)
    span = int(np.ceil(N.max())) * 2 + 4
    rays = []
    for j in range(-span, span):
        for k in range(-span, span):
            p0, v, _ = line(n, N, j, k)
            if clip_box(p0, v, np.zeros(3), N) is not None:
                rays.append((j, k))
    return rays


def rk4_segment(I0, kap, src, L, nsub=64):
    """Integrate dI/dl = kap (src - I) over [0, L]; return exit I and the
    Simpson average of I and of I0 exp(-kap l) over the segment."""
    hstep = L / nsub
    f = lambda I: kap * (src - I)
    Is = [I0]
    I = I0
    for _ in range(nsub):
        k1 = f(I)
        k2 = f(I + 0.5 * hstep * k1)
        k3 = f(I + 0.5 * hstep * k2)
        k4 = f(I + hstep * k3)
        I = I + hstep / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        Is.append(I)
    Is = np.array(Is)
    wts = np.ones(nsub + 1)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    avg_total = (wts * Is).sum() / (3.0 * nsub)
    ls = np.linspace(0.0, L, nsub + 1)
    avg_in = (wts * I0 * np.exp(-kap * ls)).sum() / (3.0 * nsub)
    return I, avg_in, avg_total


def _gl(npts=32):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w       # nodes and weights on [0, 1]


def bf_sweep(kappa, S, dirs, I_bc=0.0, h=1.0, method="rk4", nsub=64):
    """Brute-force sweep of one bin on a tiny mesh.

    kappa, S: (nz, ny, nx) float64.  method "rk4" integrates the transfer
    equation numerically through piecewise-constant cells; method "uniform"
    requires constant kappa and S and uses the analytic solution
    I(l) = I_bc e^{-kappa l} + S (1 - e^{-kappa l}) with Gauss-Legendre averages.

    Returns J_in, J_exact (nz, ny, nx) and exit_sum (N_d,), from the
    definitions: per (direction, cell) the optical-depth-weighted mean of the
    path-averaged incoming intensity (path-length weights where kappa = 0),
    and the path-length-weighted mean of the path-averaged total intensity.
    """
    shape = kappa.shape
    ncell = kappa.size
    kf = kappa.ravel()
    sf = S.ravel()
    J_in = np.zeros(ncell)
    J_ex = np.zeros(ncell)
    exits = np.zeros(len(dirs))
    xg, wg = _gl()
    if method == "uniform":
        k0 = float(kf[0])
        s0 = float(sf[0])
        assert np.all(kf == k0) and np.all(sf == s0)
    for d, n in enumerate(dirs):
        num = np.zeros(ncell)
        den = np.zeros(ncell)
        exn = np.zeros(ncell)
        exd = np.zeros(ncell)
        for (j, k) in lattice_rays(n, shape):
            chords, w = ray_chords(n, shape, j, k)
            I = I_bc
            l_entry = chords[0][1] if chords else 0.0
            for cc, sa, sb in chords:
                L = (sb - sa) * h / w
                kap, src = kf[cc], sf[cc]
                if method == "rk4":
                    I_out, avg_in, avg_tot = rk4_segment(I, kap, src, L, nsub)
                else:
                    l0 = (sa - l_entry) * h / w
                    ll = l0 + xg * L
                    I_l = I_bc * np.exp(-k0 * ll) + s0 * (1 - np.exp(-k0 * ll))
                    I_in0 = I_bc * np.exp(-k0 * l0) + s0 * (1 - np.exp(-k0 * l0))
                    avg_tot = float(np.sum(wg * I_l))
                    avg_in = float(np.sum(wg * I_in0 * np.exp(-k0 * xg * L)))
                    lx = l0 + L
                    I_out = I_bc * np.exp(-k0 * lx) + s0 * (1 - np.exp(-k0 * lx))
                wt = kap * L if kap > 0 else L
                num[cc] += wt * avg_in
                den[cc] += wt
                exn[cc] += L * avg_tot
                exd[cc] += L
                I = I_out
            if chords:
                exits[d] += I - I_bc
        J_in += num / den
        J_ex += exn / exd
    nd = len(dirs)
    return (J_in / nd).reshape(shape), (J_ex / nd).reshape(shape), exits
