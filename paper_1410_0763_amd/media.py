"""Seeded synthetic media for the diffuse-radiation sweep.

This module only draws inputs: absorption coefficients, source functions and
the shapes/sizes of the workloads.  It contains none of the transfer
arithmetic, so the CPU oracle and the GPU path can both be fed from it
without sharing any of the method's code.

Every field is returned as float32 arrays of shape (nbins, nz, ny, nx)
(x fastest).  The oracle receives the same float32 values widened to float64,
so the two sides see identical inputs.

Recipes (all seeded with numpy PCG64):

* ``uniform_random``: kappa ~ U[0.05, 2], S ~ U[0, 1] per cell (16^3 case).
* ``lognormal_density``: a periodic Gaussian random field g with power
  spectrum P(k) ~ k^-3 (k = 0 removed, unit variance) and n = exp(s g - s^2/2),
  which has mean 1.
* ``clumpy_medium``: density n lognormal, neutral fraction x_HI ~ U[0, 1],
  kappa = kappa0 * n * x_HI, recombination-like source S ~ n^2 (1 - x_HI)
  normalised to mean 1, optional dense spheres multiplying kappa by 100, and
  frequency bins nu_b/nu_0 = 1 + b/4 with kappa_b = kappa (nu_b/nu_0)^-3,
  S_b = S, rate weights g_b = (nu_b/nu_0)^-4 / nbins and heating weights
  g_b (1 - nu_0/nu_b + 1/20) (of J_in) and g_b / 20 (of S), synthetic values
  of the shape of eq heat_diff's per-bin integrals.
"""
from __future__ import annotations

import dataclasses
import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_random_field(shape, seed: int, slope: float = -3.0) -> np.ndarray:
    """Periodic Gaussian field on the mesh grid with P(k) ~ k^slope, zero mean
    and unit variance (float64, shape (nz, ny, nx))."""
    nz, ny, nx = shape
    rng = _rng(seed)
    white = rng.standard_normal((nz, ny, nx))
    fk = np.fft.rfftn(white)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    amp = np.zeros_like(k2)
    nz_mask = k2 > 0
    amp[nz_mask] = k2[nz_mask] ** (slope / 4.0)  # sqrt(P) = k^(slope/2)
    g = np.fft.irfftn(fk * amp, s=(nz, ny, nx), axes=(0, 1, 2))
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def lognormal_density(shape, sigma_ln: float, seed: int) -> np.ndarray:
    g = gaussian_random_field(shape, seed)
    return np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)


def add_spheres(field: np.ndarray, count: int, rmin: float, rmax: float,
                factor: float, seed: int) -> np.ndarray:
    """Multiply ``field`` by ``factor`` inside ``count`` spheres with radius
    ~ U[rmin, rmax] cells and centres uniform in the box."""
    nz, ny, nx = field.shape
    rng = _rng(seed)
    out = field.copy()
    z = np.arange(nz)[:, None, None] + 0.5
    y = np.arange(ny)[None, :, None] + 0.5
    x = np.arange(nx)[None, None, :] + 0.5
    mask = np.zeros(field.shape, dtype=bool)
    for _ in range(count):
        r = rng.uniform(rmin, rmax)
        cz, cy, cx = rng.uniform(0, nz), rng.uniform(0, ny), rng.uniform(0, nx)
        z0, z1 = max(0, int(cz - r) - 1), min(nz, int(cz + r) + 2)
        y0, y1 = max(0, int(cy - r) - 1), min(ny, int(cy + r) + 2)
        x0, x1 = max(0, int(cx - r) - 1), min(nx, int(cx + r) + 2)
        d2 = ((z[z0:z1] - cz) ** 2 + (y[:, y0:y1] - cy) ** 2 + (x[:, :, x0:x1] - cx) ** 2)
        mask[z0:z1, y0:y1, x0:x1] |= d2 <= r * r
    out[mask] *= factor
    return out


@dataclasses.dataclass
class Medium:
    """One synthetic workload: float32 fields plus sweep parameters."""
    name: str
    kappa: np.ndarray          # (nbins, nz, ny, nx) float32
    S: np.ndarray              # (nbins, nz, ny, nx) float32
    nside: int
    gamma_w: np.ndarray        # (nbins,) float32
    cell_size: float = 1.0
    I_bc: float = 0.0
    density: np.ndarray | None = None   # (nz, ny, nx) float32, when defined
    x_hi: np.ndarray | None = None      # (nz, ny, nx) float32, when defined
    heat_in: np.ndarray | None = None   # (nbins,) heating weights of J_in, when defined
    heat_src: np.ndarray | None = None  # (nbins,) heating weights of S, when defined

    @property
    def shape(self):
        return self.kappa.shape[1:]

    @property
    def nbins(self):
        return self.kappa.shape[0]


def uniform_random(shape=(16, 16, 16), nside=1, seed=11, kmin=0.05, kmax=2.0,
                   nbins=1) -> Medium:
    rng = _rng(seed)
    kappa = rng.uniform(kmin, kmax, size=(nbins,) + tuple(shape))
    S = rng.uniform(0.0, 1.0, size=(nbins,) + tuple(shape))
    return Medium("uniform_random", kappa.astype(np.float32), S.astype(np.float32),
                  nside, np.ones(nbins, np.float32))


def clumpy_medium(shape, nside, sigma_ln, seed, kappa0=0.5, nbins=1,
                  spheres=0, sphere_r=(4.0, 12.0), name="clumpy") -> Medium:
    """Lognormal density, x_HI ~ U[0,1], kappa = kappa0 n x_HI, S ~ n^2 (1 - x_HI)
    (mean 1), optional opaque spheres, nbins frequency bins."""
    n = lognormal_density(shape, sigma_ln, seed)
    rng = _rng(seed + 1)
    x_hi = rng.uniform(0.0, 1.0, size=shape)
    kap = kappa0 * n * x_hi
    if spheres:
        kap = add_spheres(kap, spheres, sphere_r[0], sphere_r[1], 100.0, seed + 2)
    src = n * n * (1.0 - x_hi)
    src = src / src.mean()
    nu = 1.0 + np.arange(nbins) / 4.0
    kappa = np.stack([kap * nu[b] ** -3.0 for b in range(nbins)])
    S = np.stack([src for _ in range(nbins)])
    gw = (nu ** -4.0) / nbins
    return Medium(name, kappa.astype(np.float32), S.astype(np.float32), nside,
                  gw.astype(np.float32), density=n.astype(np.float32),
                  x_hi=x_hi.astype(np.float32),
                  heat_in=(gw * (1.0 - 1.0 / nu + 0.05)).astype(np.float32),
                  heat_src=(gw * 0.05).astype(np.float32))


# ---- the five workloads -------------------------------------------------

def plain_16(seed=11) -> Medium:
    """16^3, kappa ~ U[0.05, 2], S ~ U[0, 1], nside 1, one bin."""
    return uniform_random((16, 16, 16), nside=1, seed=seed)


def plain_64(seed=22) -> Medium:
    """64^3 lognormal (sigma_ln = 1), kappa = 0.5 n x_HI, S ~ n^2 (1 - x_HI), nside 4."""
    return clumpy_medium((64, 64, 64), nside=4, sigma_ln=1.0, seed=seed, name="plain_64")


def plain_256(seed=33) -> Medium:
    """256^3 lognormal (sigma_ln = 1.5) + 64 spheres (kappa x 100), nside 8, 4 bins."""
    return clumpy_medium((256, 256, 256), nside=8, sigma_ln=1.5, seed=seed, nbins=4,
                         spheres=64, name="plain_256")


def batch_shapes(count=48, seed=4000):
    """Uneven mesh shapes (each side in [32, 128], about a third cubes), nside in
    {2, 4, 8} and 1-4 frequency bins per mesh."""
    out = []
    for i in range(count):
        rng = _rng(seed + i)
        if rng.uniform() < 1.0 / 3.0:
            s = int(rng.integers(32, 129))
            shape = (s, s, s)
        else:
            shape = tuple(int(v) for v in rng.integers(32, 129, size=3))
        nside = int(rng.choice([2, 4, 8]))
        nbins = int(rng.integers(1, 5))
        out.append((shape, nside, nbins))
    return out


def batch_media(count=48, seed=4000, scale=1.0):
    """The uneven batch: one lognormal medium per mesh.  ``scale`` < 1 shrinks
    every side (for quick tests) while keeping the mix."""
    media = []
    for i, (shape, nside, nbins) in enumerate(batch_shapes(count, seed)):
        if scale != 1.0:
            shape = tuple(max(4, int(round(v * scale))) for v in shape)
        media.append(clumpy_medium(shape, nside=nside, sigma_ln=1.0, seed=seed + 100 + i,
                                   nbins=nbins, name=f"batch_{i}"))
    return media


@dataclasses.dataclass
class PointSources:
    """Point sources in a medium: positions (nsrc, 3) as (x, y, z) in cell
    units, photon rates Q (nsrc, nbins), energies above threshold e (nbins,)
    and the absorber density n_abs (nz, ny, nx), all float64 except n_abs."""
    medium: Medium
    pos: np.ndarray
    Q: np.ndarray
    e: np.ndarray
    n_abs: np.ndarray


def point_sources(shape=(128, 128, 128), nsrc=16, nbins=4, seed=7000, spheres=16) -> PointSources:
    """The point-source workload: a lognormal medium (sigma_ln = 1.5) with
    opaque spheres and nbins bins (kappa_b = kappa0 n x_HI nu_b^-3, x 100 in
    the spheres; the absorber density is kappa_0 / kappa0, i.e. n x_HI with
    the spheres' factor, and the cross-section kappa0 nu_b^-3), nsrc
    sources at uniform random positions, photon rates Q_b ~ nu_b^-2 times a
    log-uniform luminosity per source, and energies above threshold
    e_b = nu_b - 1 + 1/8 (units of the threshold energy)."""
    med = clumpy_medium(shape, nside=1, sigma_ln=1.5, seed=seed, nbins=nbins, spheres=spheres,
                        name=f"point_{shape[0]}")
    rng = _rng(seed + 50)
    nz, ny, nx = shape
    pos = rng.uniform(0.0, 1.0, size=(nsrc, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    nu = 1.0 + np.arange(nbins) / 4.0
    lum = 10.0 ** rng.uniform(-1.0, 1.0, size=nsrc)
    Q = lum[:, None] * nu[None, :] ** -2.0
    e = nu - 1.0 + 0.125
    n_abs = (med.kappa[0].astype(np.float64) / 0.5).astype(np.float32)
    return PointSources(med, pos, Q, e, n_abs)


def surrogate_medium(i: int, train=True, shape=(128, 128, 128)) -> Medium:
    """Field i of the surrogate set: lognormal (sigma_ln = 1.5) + 16 spheres, one bin."""
    seed = (5000 if train else 6000) + i
    return clumpy_medium(shape, nside=16, sigma_ln=1.5, seed=seed, spheres=16,
                         name=f"surrogate_{'train' if train else 'test'}_{i}")
