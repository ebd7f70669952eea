"""Pins of the chemistry and energy oracle (oracle/chem.py; Appendices B-D):
closed forms of the backward-difference update and of the implicit energy
equation, photo-ionisation equilibrium, the continuum limits of pure
photo-ionisation and pure recombination, the chemical timestep formula,
table interpolation and conservation.  CPU only."""
import math

import numpy as np
import pytest

from oracle import chem as C


def _p(**kw):
    tables = {k: kw.pop(k) for k in ("alpha", "k_ci", "cool_I", "cool_II") if k in kw}
    p = C.default_params(**tables)
    p.update(kw)
    return p


def _const(v, n=61):
    return np.full(n, float(v))


def test_interpolation_exact_at_nodes_linear_between_clamped_outside():
    p = C.default_params()
    tab = np.arange(61, dtype=np.float64) ** 2
    for i in (0, 7, 60):
        T = 10.0 ** (p["logT_min"] + i * p["dlogT"])
        assert C.interp(tab, p["logT_min"], p["dlogT"], T) == pytest.approx(tab[i], rel=1e-12, abs=1e-12)
    T = 10.0 ** (p["logT_min"] + 7.25 * p["dlogT"])
    assert C.interp(tab, p["logT_min"], p["dlogT"], T) == pytest.approx(0.75 * 49 + 0.25 * 64, rel=1e-12)
    assert C.interp(tab, p["logT_min"], p["dlogT"], 1e-5) == tab[0]
    assert C.interp(tab, p["logT_min"], p["dlogT"], 1e12) == tab[-1]


def test_single_substep_is_the_backward_difference_formula():
    """One sub-step (max_sub = 0: the whole step at once) of pure
    photo-ionisation: n_HI' = n_HI / (1 + Gamma dt) exactly (C = 0)."""
    p = _p(max_sub=0)
    for G, dt in ((0.3, 2.0), (5.0, 0.01), (1e-3, 1e3)):
        x, u, _, ns = C.step_cell(1.0, 1.0, G, 0.0, 0.8, 1e4, dt, p)
        assert ns == 1
        assert x == pytest.approx(0.8 / (1.0 + G * dt), rel=1e-14)


@pytest.mark.parametrize("G,dt", [(1.0, 1.0), (0.5, 3.0)])
def test_photoionisation_converges_to_exponential_decay(G, dt):
    """With the paper's sub-step rule the neutral fraction approaches the
    solution x0 e^{-Gamma t} of dn_HI/dt = -Gamma n_HI, and the error falls
    tenfold when both timestep factors are ten times smaller (first-order
    backward differences, in the asymptotic range)."""
    exact = 0.9 * math.exp(-G * dt)
    errs = []
    for scale in (1.0, 0.1, 0.01):
        p = _p(eps_e=0.2 * scale, eps_HI=0.002 * scale)
        x, _, _, _ = C.step_cell(1.0, 1.0, G, 0.0, 0.9, 1e4, dt, p)
        errs.append(abs(x - exact) / exact)
    assert errs[0] < 0.2
    assert 8.0 < errs[1] / errs[2] < 12.0


def test_recombination_converges_to_the_analytic_decay():
    """Gamma = 0, constant alpha, no collisional ionisation: n_HII(t) =
    n0 / (1 + alpha n0 t); first-order convergence in the timestep factors."""
    a, n0, dt = 2.0, 1.0, 3.0
    exact = n0 / (1.0 + a * n0 * dt)
    errs = []
    for scale in (1.0, 0.1, 0.01):
        p = _p(alpha=_const(a), eps_e=0.2 * scale, eps_HI=0.002 * scale)
        x, _, _, _ = C.step_cell(1.0, 1.0, 0.0, 0.0, 1.0 - n0, 1e4, dt, p)
        errs.append(abs((1.0 - x) - exact) / exact)
    assert errs[0] < 0.2
    assert 8.0 < errs[1] / errs[2] < 12.0


@pytest.mark.parametrize("a,G,nH", [(1.0, 0.5, 1.0), (3e-2, 4.0, 2.5), (10.0, 0.01, 0.3)])
def test_photoionisation_equilibrium(a, G, nH):
    """Constant alpha and Gamma, no collisions, no heating or cooling: after a
    long step x_HI is the root of alpha n_H (1 - x)^2 = Gamma x in [0, 1] (to
    the paper's iteration tolerance 1e-3)."""
    A = a * nH
    x_eq = ((2 * A + G) - math.sqrt((2 * A + G) ** 2 - 4 * A * A)) / (2 * A)
    for x0 in (0.999, 0.001):
        p = _p(alpha=_const(a))
        x, _, _, _ = C.step_cell(nH, 1.0, G, 0.0, x0, 1e4, 1e4 / G, p)
        assert abs(x - x_eq) <= 2e-3 * max(x_eq, 1.0 - x_eq)


def test_heating_only_is_exact():
    """Fixed species (no reactions) and photo-heating only: u(dt) = u0 + dt
    Heat n_HI / rho exactly, whatever the sub-steps."""
    p = _p()
    nH, x0, rho, H, u0, dt = 2.0, 0.4, 1.7, 3.0, 50.0, 0.9
    x, u, _, _ = C.step_cell(nH, rho, 0.0, H, x0, u0, dt, p)
    assert x == x0
    assert u == pytest.approx(u0 + dt * H * x0 * nH / rho, rel=1e-13)


def test_constant_cooling_is_linear_down_to_the_floor():
    """Fixed species, cooling coefficients independent of T, no heating: u
    falls linearly at Lambda / rho and stops at the floor (the lowest tabulated
    temperature)."""
    nH, x0, rho, LI, LII = 1.0, 0.3, 1.0, 0.2, 0.5
    p = _p(cool_I=_const(LI), cool_II=_const(LII))
    ne = (1 - x0) * nH
    lam = ne * (LI * x0 * nH + LII * (1 - x0) * nH)
    u0, dt = 1e4, 100.0
    _, u, _, _ = C.step_cell(nH, rho, 0.0, 0.0, x0, u0, dt, p)
    assert u == pytest.approx(u0 - dt * lam / rho, rel=1e-12)
    floor = 10.0 ** p["logT_min"] / p["T_per_u"]
    _, u, _, _ = C.step_cell(nH, rho, 0.0, 0.0, x0, u0, 1e6, p)
    assert u == floor


def test_chemical_timestep_formula():
    """dt_chem = eps_e |n_e / n_e'| + eps_HI |n_HI / n_HI'| at a hand-made state."""
    p = _p(alpha=_const(2.0), k_ci=_const(0.5))
    nH, x, G = 1.0, 0.25, 3.0
    nHI, ne = x * nH, (1 - x) * nH
    dHI = 2.0 * ne * ne - (0.5 * ne + G) * nHI
    want = 0.2 * abs(ne / dHI) + 0.002 * abs(nHI / dHI)
    assert C.chem_timestep(nH, nHI, 1e4, G, p) == pytest.approx(want, rel=1e-14)
    # a rate of zero makes its term infinite; an equilibrium state has no limit
    assert C.chem_timestep(nH, nH, 1e4, 0.0, _p()) == math.inf


def test_temperature_and_mean_mass():
    p = _p(T_per_u=2.0)
    assert C.temperature(100.0, 0.0, p) == 200.0       # neutral
    assert C.temperature(100.0, 1.0, p) == 100.0       # ionised: twice the particles


def test_conservation_and_bounds_on_random_states():
    rng = np.random.default_rng(8)
    T = np.linspace(1.0, 9.0, 61)
    p = _p(alpha=2e-3 * (10 ** T / 1e4) ** -0.7, k_ci=1e-3 * np.exp(-10 ** (5.2 - T)),
           cool_I=1e-4 * np.exp(-10 ** (5.0 - T)), cool_II=1e-6 * (10 ** T) ** 0.5, T_per_u=1e2)
    n = 40
    nH = rng.lognormal(0, 1, n)
    xo, uo, tc, ns = C.step(nH, nH, rng.uniform(0, 2, n), rng.uniform(0, 5, n), rng.uniform(0, 1, n),
                            rng.uniform(1, 1e3, n), 0.5, p)
    assert np.all((xo >= 0) & (xo <= 1)) and np.all(uo >= 10.0 ** p["logT_min"] / p["T_per_u"])
    assert np.all(ns >= 1) and np.all(tc > 0)


@pytest.mark.parametrize("a,k", [(1.0, 0.25), (0.1, 3.0)])
def test_collisional_ionisation_equilibrium(a, k):
    """No radiation, constant alpha and k_ci: recombination balances collisional
    ionisation when alpha n_HII = k_ci n_HI, i.e. x_HI = alpha / (alpha + k_ci)
    whatever the density."""
    x_eq = a / (a + k)
    for nH, x0 in ((1.0, 0.5), (7.0, 0.05), (0.2, 0.9)):
        p = _p(alpha=_const(a), k_ci=_const(k))
        x, _, _, _ = C.step_cell(nH, 1.0, 0.0, 0.0, x0, 1e4, 200.0 / (a * nH), p)
        assert abs(x - x_eq) <= 2e-3 * max(x_eq, 1.0 - x_eq)
