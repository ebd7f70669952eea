"""FP64 CPU oracle of the chemistry and energy update that follows each
radiative-transfer step (Appendices B, C and D of Tanaka et al.,
arXiv:1410.0763), for a hydrogen-only network.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the HIP kernel
art_chem_step; the product path never calls it.  It shares no code with the
library.  Plain per-cell Python loops in float64 (small inputs only).

Readings (the paper cites its rate fits without printing them):

* C1 species.  HI and HII only (n_e = n_HII); x_HI = n_HI / n_H.
* C2 rates.  Caller tables on a uniform grid of log10 T: alpha (radiative
  recombination of HII, per n_e n_HII), k_ci (collisional ionisation of HI,
  per n_e n_HI), cool_I and cool_II (cooling per n_e n_HI and per n_e n_HII:
  collisional ionisation and excitation; recombination and bremsstrahlung),
  each interpolated linearly in log10 T and held at the end values outside
  the grid.  Photo-ionisation Gamma and photo-heating Heat per HI atom come
  from the radiative transfer and are constant during the step (the transfer
  equation is static).
* C3 temperature.  T = T_per_u u / (1 + x_e), x_e = n_HII / n_H (mean mass
  per particle of ionised hydrogen); u is floored at the grid's lowest
  temperature for a neutral gas, u_floor = 10^logT_min / T_per_u.
* C4 the step (Appendix D).  Sub-steps h = min(dt_chem, dt - t) with
  dt_chem = eps_e |n_e / dn_e/dt| + eps_HI |n_HI / dn_HI/dt| at the sub-step's
  start (a term whose rate is 0 is infinite); after max_sub sub-steps the
  rest of dt is taken at once.  Within a sub-step the update is iterated
  until |n_e^(i) - n_e^(i-1)| < eps n_e^(i) and |u^(i) - u^(i-1)| < eps u^(i)
  (eps = 1e-3), at most max_iter times:
    - Appendix B: n_HI' = (C h + n_HI) / (1 + D h) with C = alpha n_e' n_HII'
      and D = k_ci n_e' + Gamma at the advanced time.  With hydrogen alone
      n_e' = n_HII' = n_H - n_HI', so at the temperature T' of the latest
      iterate this is a quadratic in n_HI'; its root in [0, n_H] is taken
      exactly (iterating n_HI' = (C h + n_HI) / (1 + D h) on the densities is
      unstable once alpha n_H h is large);
    - Appendix C: u' solves u' = u + h (Heat n_HI' - Lambda(n', u')) / rho,
      Lambda = n_e' (cool_I(T) n_HI' + cool_II(T) n_HII'), found by 64
      bisection halvings on [u_floor, max(u_floor, u + h Heat n_HI' / rho)]
      (u_floor when the residual there is already >= 0).
* C5 outputs.  x_HI, u after dt; dt_chem at the final state (the chemical
  timestep of Appendix D from which the next radiative step is set).
"""
from __future__ import annotations

import math

import numpy as np


def interp(table, logT_min, dlogT, T):
    """Linear interpolation of a table on the uniform log10 T grid (C2)."""
    n = len(table)
    lt = math.log10(max(T, 1e-300))
    s = (lt - logT_min) / dlogT
    if s <= 0.0:
        return float(table[0])
    if s >= n - 1:
        return float(table[n - 1])
    i = int(math.floor(s))
    f = s - i
    return float(table[i]) * (1.0 - f) + float(table[i + 1]) * f


def temperature(u, x_e, p):
    """C3: T from the specific internal energy and the ionised fraction."""
    return p["T_per_u"] * u / (1.0 + x_e)


def rates(nH, nHI, u, Gamma, p):
    """dn_HI/dt and dn_e/dt at a state (Appendix B, eq app_chem)."""
    nHII = nH - nHI
    ne = nHII
    T = temperature(u, nHII / nH, p)
    a = interp(p["alpha"], p["logT_min"], p["dlogT"], T)
    k = interp(p["k_ci"], p["logT_min"], p["dlogT"], T)
    dHI = a * ne * nHII - (k * ne + Gamma) * nHI
    return dHI, -dHI


def chem_timestep(nH, nHI, u, Gamma, p):
    """Appendix D: eps_e |n_e / n_e'| + eps_HI |n_HI / n_HI'|."""
    dHI, de = rates(nH, nHI, u, Gamma, p)
    ne = nH - nHI
    t1 = math.inf if de == 0.0 else p["eps_e"] * abs(ne / de)
    t2 = math.inf if dHI == 0.0 else p["eps_HI"] * abs(nHI / dHI)
    return t1 + t2


def energy_solve(u0, h, Heat, nH, nHI, rho, p):
    """Appendix C: implicit u' for the species n' (bisection, C4)."""
    nHII = nH - nHI
    ne = nHII
    u_floor = 10.0 ** p["logT_min"] / p["T_per_u"]

    def resid(uu):
        T = temperature(uu, nHII / nH, p)
        lam = ne * (interp(p["cool_I"], p["logT_min"], p["dlogT"], T) * nHI +
                    interp(p["cool_II"], p["logT_min"], p["dlogT"], T) * nHII)
        return uu - u0 - h * (Heat * nHI - lam) / rho

    lo = u_floor
    hi = max(u_floor, u0 + h * Heat * nHI / rho)
    if resid(lo) >= 0.0:
        return lo
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if resid(mid) >= 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def hi_advanced(nH, nHI0, h, a, k, Gamma):
    """Appendix B at fixed rate coefficients: the n_HI' in [0, n_H] with
    n_HI' (1 + (k n_e' + Gamma) h) = a n_e' n_HII' h + n_HI0, n_e' = n_HII' =
    n_H - n_HI', i.e. the smaller root of
    (k + a) h y^2 - (1 + (k + 2 a) h n_H + Gamma h) y + a h n_H^2 + n_HI0 = 0."""
    q2 = (k + a) * h
    b = 1.0 + (k + 2.0 * a) * h * nH + Gamma * h
    c = a * h * nH * nH + nHI0
    disc = max(b * b - 4.0 * q2 * c, 0.0)
    y = 2.0 * c / (b + math.sqrt(disc))
    return min(max(y, 0.0), nH)


def substep(nH, nHI, u, h, Gamma, Heat, rho, p):
    """One sub-step: the iterated BDF and implicit energy update (C4)."""
    nHI_i, u_i = nHI, u
    ne_prev = nH - nHI
    iters = 0
    for it in range(p["max_iter"]):
        iters = it + 1
        T = temperature(u_i, (nH - nHI_i) / nH, p)
        a = interp(p["alpha"], p["logT_min"], p["dlogT"], T)
        k = interp(p["k_ci"], p["logT_min"], p["dlogT"], T)
        nHI_new = hi_advanced(nH, nHI, h, a, k, Gamma)
        u_new = energy_solve(u, h, Heat, nH, nHI_new, rho, p)
        ne_new = nH - nHI_new
        done = (abs(ne_new - ne_prev) <= p["eps"] * ne_new and abs(u_new - u_i) <= p["eps"] * u_new)
        nHI_i, u_i, ne_prev = nHI_new, u_new, ne_new
        if done:
            break
    return nHI_i, u_i, iters


def step_cell(nH, rho, Gamma, Heat, xHI, u, dt, p):
    """One radiative step dt for one cell: (x_HI, u, dt_chem, substeps)."""
    if not nH > 0.0:
        return xHI, u, math.inf, 0
    nHI = xHI * nH
    t = 0.0
    nsub = 0
    while t < dt:
        if nsub >= p["max_sub"]:
            h = dt - t
        else:
            h = min(chem_timestep(nH, nHI, u, Gamma, p), dt - t)
        nHI, u, _ = substep(nH, nHI, u, h, Gamma, Heat, rho, p)
        t = t + h if h < dt - t else dt
        nsub += 1
    return nHI / nH, u, chem_timestep(nH, nHI, u, Gamma, p), nsub


def step(nH, rho, Gamma, Heat, xHI, u, dt, p):
    """All cells (1-D arrays): returns x_HI, u, dt_chem, substeps."""
    n = len(nH)
    xo, uo, tc, ns = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int64)
    for i in range(n):
        xo[i], uo[i], tc[i], ns[i] = step_cell(float(nH[i]), float(rho[i]), float(Gamma[i]),
                                              float(Heat[i]), float(xHI[i]), float(u[i]), float(dt), p)
    return xo, uo, tc, ns


def default_params(nT=61, logT_min=1.0, logT_max=9.0, **tables):
    """A parameter dict: uniform log10 T grid, tables (default all zero), the
    paper's tolerances (eps 1e-3, eps_e 0.2, eps_HI 0.002), T_per_u 1."""
    p = dict(logT_min=logT_min, dlogT=(logT_max - logT_min) / (nT - 1), T_per_u=1.0, eps=1e-3,
             eps_e=0.2, eps_HI=0.002, max_iter=100, max_sub=100000)
    for name in ("alpha", "k_ci", "cool_I", "cool_II"):
        p[name] = np.asarray(tables.get(name, np.zeros(nT)), dtype=np.float64)
    return p
