"""FP64 CPU oracle of one radiative step coupled to the chemistry and energy
update (Tanaka et al., arXiv:1410.0763): the transfer equation is static, so
the diffuse radiation field and the rate and energy equations are iterated
until the electron density and the specific energy of every cell converge
(Appendix D); the absorption coefficient and the source function of the
diffuse recombination radiation follow from the chemical state (Sect. 2.2).

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the HIP entry point
art_rt_chem_step; the product path never calls it.  It composes the sweep
oracle (`oracle.oracle.sweep`, FP64 C) and the chemistry oracle
(`oracle.chem.step`) and shares no code with the library.

Readings (the paper gives the model, not the code):

* R1 fields.  Per bin b (the paper transfers one bin at the Lyman limit;
  more bins take their own constants): kappa_b = sigma_b n_HI and
  S_b = c_b dalpha(T) n_e n_HII / n_HI, the source function
  epsilon / kappa of the rectangular recombination spectrum (Sect. 2.2:
  epsilon / (h nu) = dalpha n_e n_HII / (4 pi dnu_th) over the band, so
  c_b = h nu_0 / (4 pi sigma_b dnu_th) in the paper's units), with
  dalpha = alpha_A - alpha_B a caller table on the chemistry's log10 T grid
  and T from the chemistry's model.  n_HI is floored at x_floor n_H in both
  (the paper does not treat a fully ionised cell; with the floor such a cell
  absorbs next to nothing and emits epsilon dL along a segment, the limit of
  S (1 - e^{-kappa dL})).  Cells with n_H <= 0 have kappa = S = 0.
* R2 rates.  Gamma = sum_b g_b (J_in_b + S_b), Heat = sum_b (hin_b J_in_b +
  hsrc_b S_b) of the sweep (eqs gamma_diff and heat_diff, the frequency
  integrals folded into caller weights); g_b S_b is the on-the-spot term
  dalpha n_e n_HII / n_HI of eq gamma_diff when g_b c_b = 1.  Point sources,
  if any, add their photon-conserving rates per absorber (Sect. 2.3,
  Appendix A; `oracle.point`) for the same kappa, with the same floored
  n_HI as the absorber density.
* R3 iteration.  Iteration i (i = 1, 2, ...) builds the fields from the state
  of iteration i - 1 (iteration 0: the state at the start of the step),
  sweeps, and advances every cell from the start state over dt with those
  rates (`chem.step`: sub-steps, species and energy).  It stops when every
  cell with n_H > 0 has |n_e^(i) - n_e^(i-1)| <= eps n_e^(i) and
  |u^(i) - u^(i-1)| <= eps u^(i) (eps of the chemistry parameters), or after
  max_iter iterations (then not converged).  Returned: the state of the last
  iteration, its number, whether it converged, and the minimum chemical
  timestep over the cells at that state (the radiative step is F times it).
* R4 time stepping (Appendix D).  From t = 0 to t_end: the chemical
  timestep of the start state, with the rates of its own fields, is that of
  a step of length 0; then each radiative step is dt = min(F dt_chem_min,
  t_end - t) with dt_chem_min from the end of the previous step (a step with
  an infinite dt_chem_min takes the rest at once), until t_end or max_steps.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import chem as C
from oracle import oracle as O


def fields(nH, x, u, rp, cp):
    """R1: kappa_b and S_b (float64, shape (nbins,) + nH.shape)."""
    nH = np.asarray(nH, np.float64)
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    nb = len(rp["sigma"])
    kappa = np.zeros((nb,) + nH.shape)
    S = np.zeros((nb,) + nH.shape)
    for idx in np.ndindex(nH.shape):
        n = float(nH[idx])
        if not n > 0.0:
            continue
        nHI = n * max(float(x[idx]), rp["x_floor"])
        ne = n * (1.0 - float(x[idx]))
        T = C.temperature(float(u[idx]), ne / n, cp)
        da = C.interp(rp["dalpha"], cp["logT_min"], cp["dlogT"], T)
        for b in range(nb):
            kappa[(b,) + idx] = rp["sigma"][b] * nHI
            S[(b,) + idx] = rp["src_coef"][b] * da * ne * ne / nHI
    return kappa, S


def converged(nH, x_new, u_new, x_old, u_old, eps):
    """R3: the convergence test of Appendix D over the cells with n_H > 0."""
    ok = True
    for i in range(len(nH)):
        if not nH[i] > 0.0:
            continue
        ne_new = nH[i] * (1.0 - x_new[i])
        ne_old = nH[i] * (1.0 - x_old[i])
        if not (abs(ne_new - ne_old) <= eps * ne_new and abs(u_new[i] - u_old[i]) <= eps * u_new[i]):
            ok = False
    return ok


def step(shape, h, nH, rho, x0, u0, dt, rp, cp, max_iter, nthreads=0):
    """One coupled radiative step on a mesh of shape (nz, ny, nx), cell size h.
    nH, rho, x0, u0: float64 arrays of nz*ny*nx cells (x fastest).  Returns
    dict x, u, iterations, converged, dt_chem_min, Gamma, Heat (the last
    iteration's rates)."""
    nz, ny, nx = shape
    nH = np.asarray(nH, np.float64).reshape(-1)
    rho = np.asarray(rho, np.float64).reshape(-1)
    x_prev = np.asarray(x0, np.float64).reshape(-1).copy()
    u_prev = np.asarray(u0, np.float64).reshape(-1).copy()
    nb = len(rp["sigma"])
    it, conv = 0, False
    dtc = np.full(len(nH), math.inf)
    G = H = None
    for it in range(1, max_iter + 1):
        kappa, S = fields(nH, x_prev, u_prev, rp, cp)
        out = O.sweep(kappa.reshape(nb, nz, ny, nx), S.reshape(nb, nz, ny, nx), rp["nside"],
                      gamma_w=rp["gamma_w"], h=h, heat_in=rp["heat_in"], heat_src=rp["heat_src"],
                      nthreads=nthreads)
        G = out["Gamma"].reshape(-1)
        H = out["Heat"].reshape(-1)
        if rp.get("src_pos") is not None and len(rp["src_pos"]):
            n_abs = np.where(nH > 0.0, nH * np.maximum(x_prev, rp["x_floor"]), 0.0)
            pt = O.point(kappa.reshape(nb, nz, ny, nx), n_abs.reshape(nz, ny, nx), rp["src_pos"],
                         rp["src_Q"], rp.get("src_e"), h=h, nthreads=nthreads)
            G = G + pt["Gamma"]
            H = H + pt["Heat"]
        x_new, u_new, dtc, _ = C.step(nH, rho, G, H, x0.reshape(-1), u0.reshape(-1), dt, cp)
        conv = converged(nH, x_new, u_new, x_prev, u_prev, cp["eps"])
        x_prev, u_prev = x_new, u_new
        if conv:
            break
    return dict(x=x_prev, u=u_prev, iterations=it, converged=conv,
                dt_chem_min=float(np.min(dtc)) if len(dtc) else math.inf, Gamma=G, Heat=H)


def advance(shape, h, nH, rho, x0, u0, t_end, F, rp, cp, max_iter, max_steps, nthreads=0):
    """R4: radiative steps from 0 to t_end.  Returns dict x, u, t, steps,
    iterations, unconverged, dts (the step lengths), dt_chem_min."""
    x = np.asarray(x0, np.float64).reshape(-1).copy()
    u = np.asarray(u0, np.float64).reshape(-1).copy()
    r = step(shape, h, nH, rho, x, u, 0.0, rp, cp, max_iter, nthreads)
    dcm = r["dt_chem_min"]
    t, steps, its, unconv, dts = 0.0, 0, 0, 0, []
    while t < t_end and steps < max_steps:
        rest = t_end - t
        dt = min(F * dcm, rest) if math.isfinite(dcm) else rest
        r = step(shape, h, nH, rho, x, u, dt, rp, cp, max_iter, nthreads)
        x, u, dcm = r["x"], r["u"], r["dt_chem_min"]
        t = t + dt if dt < rest else t_end
        steps += 1
        its += r["iterations"]
        unconv += 0 if r["converged"] else 1
        dts.append(dt)
    return dict(x=x, u=u, t=t, steps=steps, iterations=its, unconverged=unconv, dts=dts, dt_chem_min=dcm)


def default_rt_params(nbins=1, nT=61, **kw):
    """Radiation parameters: sigma 1, src_coef 1, dalpha all zero, weights
    g = 1 / src_coef (the on-the-spot balance of R2), no heating, Nside 1,
    x_floor 1e-6, no point sources (src_pos (nsrc, 3) cell units, src_Q
    (nsrc, nbins) photon rates, src_e (nbins,) or None)."""
    rp = dict(sigma=[1.0] * nbins, src_coef=[1.0] * nbins, dalpha=np.zeros(nT), gamma_w=[1.0] * nbins,
              heat_in=[0.0] * nbins, heat_src=[0.0] * nbins, nside=1, x_floor=1e-6,
              src_pos=None, src_Q=None, src_e=None)
    rp.update(kw)
    return rp
