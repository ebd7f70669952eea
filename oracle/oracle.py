"""Python face of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the product path never does.  It shares no code
with the HIP implementation.

The C library marches the rays and normalises each (direction, cell) average
literally (Sect. 2.2, eqs rt / path_averaged_intensity / averaged_intensity);
the last, elementwise step of eq mean_intensity, the rate of eq gamma_diff
and the heating of eq heat_diff are written out here in numpy float64.  It
also evaluates the photon-conserving rates of point sources (Sect. 2.3 and
Appendix A), `point` and `point_pair`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP, IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_ndirs.argtypes = [ctypes.c_int]
        L.oracle_directions.argtypes = [ctypes.c_int, dp]
        L.oracle_dir_geom.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.oracle_lattice.argtypes = [ctypes.c_int] * 5 + [ip]
        L.oracle_ray_segments.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] +
                                          [ctypes.c_int] * 4 + [ip, dp, dp, ctypes.c_int])
        L.oracle_sweep.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp] +
                                   [ctypes.c_int] * 3 + [ctypes.c_double, dp, dp, dp, dp,
                                                         ctypes.c_int])
        L.oracle_cells.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp] +
                                   [ctypes.c_int] * 3 + [ctypes.c_double,
                                                         ctypes.POINTER(ctypes.c_int64),
                                                         ctypes.c_int, dp, dp, ctypes.c_int])
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_point_pair.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp,
                                                              ctypes.c_int64, dp, dp, dp, dp])
        L.oracle_point.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_int, dp, dp,
                                                         ctypes.c_int, dp, dp, dp, i64p,
                                                         ctypes.c_int, dp, dp, ctypes.c_int])
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def ndirs(nside: int) -> int:
    return 12 * nside * nside


def directions(nside: int) -> np.ndarray:
    """HEALPix RING pixel centres, shape (12 nside^2, 3)."""
    out = np.zeros((ndirs(nside), 3))
    got = lib().oracle_directions(nside, _dp(out))
    assert got == ndirs(nside)
    return out


def dir_geom(nside: int, d: int) -> dict:
    """Dominant axis a, other axes b < c, sign, w = |n_a|, slopes t_b, t_c."""
    out = np.zeros(7)
    assert lib().oracle_dir_geom(nside, d, _dp(out)) == 0
    return dict(a=int(out[0]), b=int(out[1]), c=int(out[2]), sig=int(out[3]),
                w=out[4], tb=out[5], tc=out[6])


def lattice(shape, nside: int, d: int):
    """Conservative lattice range (jlo, jhi, klo, khi), inclusive; shape=(nz,ny,nx)."""
    nz, ny, nx = shape
    r = np.zeros(4, dtype=np.int32)
    assert lib().oracle_lattice(nx, ny, nz, nside, d,
                                r.ctypes.data_as(ctypes.POINTER(ctypes.c_int))) == 0
    return tuple(int(v) for v in r)


def ray_segments(shape, nside: int, d: int, j: int, k: int, h: float = 1.0):
    """Segments of ray (j, k): (cell index, path length, entry depth) arrays."""
    nz, ny, nx = shape
    m = nx + ny + nz + 8
    cell = np.zeros(m, dtype=np.int32)
    dl = np.zeros(m)
    s0 = np.zeros(m)
    ns = lib().oracle_ray_segments(nx, ny, nz, h, nside, d, j, k,
                                   cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   _dp(dl), _dp(s0), m)
    assert ns >= 0
    return cell[:ns].copy(), dl[:ns].copy(), s0[:ns].copy()


def sweep_raw(kappa, S, nside: int, h: float = 1.0, I_bc: float = 0.0,
              d_range=None, nthreads: int = 0):
    """Raw direction sums over d in d_range (default: all directions).

    kappa, S: arrays (nbins, nz, ny, nx), converted to float64.
    Returns dict with jin_sum, ex_sum (nbins, nz, ny, nx), exit_sum (N_d, nbins),
    nseg (segments with positive length, one bin), inv_err, max_hits.
    """
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    if kappa.ndim == 3:
        kappa = kappa[None]
        S = S[None]
    nb, nz, ny, nx = kappa.shape
    assert S.shape == kappa.shape
    nd = ndirs(nside)
    d0, d1 = d_range if d_range is not None else (0, nd)
    jin = np.zeros_like(kappa)
    ex = np.zeros_like(kappa)
    exit_sum = np.zeros((nd, nb))
    stats = np.zeros(3)
    rc = lib().oracle_sweep(nx, ny, nz, float(h), nb, _dp(kappa), _dp(S), nside, d0, d1,
                            float(I_bc), _dp(jin), _dp(ex), _dp(exit_sum), _dp(stats),
                            int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_sweep failed ({rc})")
    return dict(jin_sum=jin, ex_sum=ex, exit_sum=exit_sum, nseg=int(stats[0]),
                inv_err=float(stats[1]), max_hits=int(stats[2]), nd=nd, d_range=(d0, d1))


def heating(J_in, S, heat_in=None, heat_src=None):
    """Diffuse photo-heating rate with the frequency integrals of eq heat_diff
    folded into per-bin weights (reading Q12): sum_b heat_in_b J_in_b +
    heat_src_b S_b over the leading (bin) axis; missing weights are 0."""
    nb = J_in.shape[0]
    hi = np.zeros(nb) if heat_in is None else np.asarray(heat_in, dtype=np.float64)
    hs = np.zeros(nb) if heat_src is None else np.asarray(heat_src, dtype=np.float64)
    return np.tensordot(hi, J_in, axes=(0, 0)) + np.tensordot(hs, S, axes=(0, 0))


def sweep(kappa, S, nside: int, gamma_w=None, h: float = 1.0, I_bc: float = 0.0,
          nthreads: int = 0, heat_in=None, heat_src=None):
    """All outputs of one full sweep, float64.

    J_in    = (1/N_d) sum_d Ibar^{ave,in}          (eq mean_intensity, J^in)
    J       = J_in + S                              (eq mean_intensity)
    J_exact = J_in + S (1/N_d) sum_d <1 - phi>     (reading Q4)
    Gamma   = sum_b g_b (J_in_b + S_b)              (eq gamma_diff, reading Q5)
    Heat    = sum_b hin_b J_in_b + hsrc_b S_b       (eq heat_diff, reading Q12)
    """
    raw = sweep_raw(kappa, S, nside, h=h, I_bc=I_bc, nthreads=nthreads)
    S64 = np.asarray(S, dtype=np.float64)
    if S64.ndim == 3:
        S64 = S64[None]
    nd = raw["nd"]
    J_in = raw["jin_sum"] / nd
    J = J_in + S64
    J_exact = J_in + S64 * (raw["ex_sum"] / nd)
    g = np.ones(S64.shape[0]) if gamma_w is None else np.asarray(gamma_w, dtype=np.float64)
    Gamma = np.tensordot(g, J_in + S64, axes=(0, 0))
    Heat = heating(J_in, S64, heat_in, heat_src)
    return dict(J_in=J_in, J=J, J_exact=J_exact, Gamma=Gamma, Heat=Heat, exit_sum=raw["exit_sum"],
                nseg=raw["nseg"], inv_err=raw["inv_err"], max_hits=raw["max_hits"], nd=nd)


def cells(kappa, S, nside: int, cell_idx, gamma_w=None, h: float = 1.0, I_bc: float = 0.0,
          d_range=None, nthreads: int = 0, heat_in=None, heat_src=None):
    """The outputs of `sweep` at chosen cells only, float64.

    cell_idx: flat x-fastest cell indices.  Each cell's direction sums are
    formed from the rays that cross it, each marched from its entry up to
    the cell (same definitions as the full sweep).  Returns dict with
    jin_sum, ex_sum (nbins, ncells) over d_range, and, for the full
    direction set, J_in, J, J_exact (nbins, ncells), Gamma and Heat (ncells,).
    """
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    if kappa.ndim == 3:
        kappa = kappa[None]
        S = S[None]
    nb, nz, ny, nx = kappa.shape
    idx = np.ascontiguousarray(cell_idx, dtype=np.int64).ravel()
    nd = ndirs(nside)
    d0, d1 = d_range if d_range is not None else (0, nd)
    jin = np.zeros((nb, idx.size))
    ex = np.zeros((nb, idx.size))
    rc = lib().oracle_cells(nx, ny, nz, float(h), nb, _dp(kappa), _dp(S), nside, d0, d1,
                            float(I_bc), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            idx.size, _dp(jin), _dp(ex), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_cells failed ({rc})")
    out = dict(jin_sum=jin, ex_sum=ex, nd=nd, d_range=(d0, d1))
    if (d0, d1) == (0, nd):
        S_c = S.reshape(nb, -1)[:, idx]
        J_in = jin / nd
        out["J_in"] = J_in
        out["J"] = J_in + S_c
        out["J_exact"] = J_in + S_c * (ex / nd)
        g = np.ones(nb) if gamma_w is None else np.asarray(gamma_w, dtype=np.float64)
        out["Gamma"] = np.tensordot(g, J_in + S_c, axes=(0, 0))
        out["Heat"] = heating(J_in, S_c, heat_in, heat_src)
    return out


def _kappa4(kappa):
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    return kappa[None] if kappa.ndim == 3 else kappa


def point_pair(kappa, p, cell: int, h: float = 1.0):
    """Optical depths of one (source, cell) pair: dict tau, dtau (nbins,) and
    r_in, r_out (cell units) of the line from p through the cell's centre."""
    kappa = _kappa4(kappa)
    nb, nz, ny, nx = kappa.shape
    pp = np.ascontiguousarray(p, dtype=np.float64)
    tau = np.zeros(nb)
    dtau = np.zeros(nb)
    rin = ctypes.c_double()
    rout = ctypes.c_double()
    rc = lib().oracle_point_pair(nx, ny, nz, float(h), nb, _dp(kappa), _dp(pp), int(cell),
                                 _dp(tau), _dp(dtau), ctypes.byref(rin), ctypes.byref(rout))
    if rc != 0:
        raise ValueError(f"oracle_point_pair failed ({rc})")
    return dict(tau=tau, dtau=dtau, r_in=rin.value, r_out=rout.value)


def point(kappa, n_abs, pos, Q, e=None, h: float = 1.0, cell_idx=None, nthreads: int = 0):
    """Photon-conserving rates per absorber from point sources (Sect. 2.3,
    Appendix A), float64.

    kappa (nbins, nz, ny, nx) or (nz, ny, nx) per unit length; n_abs (nz, ny,
    nx) absorber density; pos (nsrc, 3) source positions (x, y, z) in cell
    units; Q (nsrc, nbins) photon rates; e (nbins,) energy per absorbed photon
    above threshold or None.  Returns dict Gamma, Heat at cell_idx (flat,
    x-fastest) or, if None, over the whole mesh (flat)."""
    kappa = _kappa4(kappa)
    nb, nz, ny, nx = kappa.shape
    n = np.ascontiguousarray(n_abs, dtype=np.float64).reshape(-1)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(pos.shape[0], nb)
    ev = None if e is None else np.ascontiguousarray(e, dtype=np.float64).reshape(nb)
    if cell_idx is None:
        idx = None
        m = nx * ny * nz
    else:
        idx = np.ascontiguousarray(cell_idx, dtype=np.int64).ravel()
        m = idx.size
    G = np.zeros(m)
    H = np.zeros(m)
    rc = lib().oracle_point(nx, ny, nz, float(h), nb, _dp(kappa), _dp(n), pos.shape[0], _dp(pos),
                            _dp(Q), _dp(ev),
                            None if idx is None else idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            m, _dp(G), _dp(H), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_point failed ({rc})")
    return dict(Gamma=G, Heat=H)
