"""Pins of the coupled transfer-chemistry oracle (oracle/rtchem.py; Sect. 2.2
and Appendix D): without radiation the step is one chemistry step and stops
at the second iteration; with dt = 0 it stops at the first; in the interior
of an optically thick uniform medium the diffuse recombination photons are
absorbed where they are emitted, so the converged ionisation balance is the
case-B one (alpha_B = alpha_A - dalpha), not the case-A one of the
chemistry alone; a converged state is a fixed point of one more iteration;
the fields reproduce the on-the-spot term of eq gamma_diff.  CPU only."""
import math

import numpy as np
import pytest

from oracle import chem as C
from oracle import rtchem as RC


def _const(v, n=61):
    return np.full(n, float(v))


def _medium(shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    nH = rng.uniform(0.5, 2.0, n)
    x = rng.uniform(0.05, 0.95, n)
    u = rng.uniform(50.0, 500.0, n)
    return nH, nH * 1.1, x, u


def test_without_radiation_the_step_is_one_chemistry_step():
    """sigma = 0 and dalpha = 0: kappa = S = 0, so Gamma = Heat = 0 whatever
    the state; the first iteration is the chemistry step with no radiation
    and the second repeats it exactly."""
    shape = (3, 4, 5)
    nH, rho, x0, u0 = _medium(shape, 1)
    cp = C.default_params(alpha=_const(1.0), k_ci=_const(0.1), cool_II=_const(1e-3))
    rp = RC.default_rt_params(sigma=[0.0])
    r = RC.step(shape, 1.0, nH, rho, x0, u0, 0.7, rp, cp, max_iter=10)
    xr, ur, tc, _ = C.step(nH, rho, np.zeros_like(nH), np.zeros_like(nH), x0, u0, 0.7, cp)
    assert r["iterations"] == 2 and r["converged"]
    assert np.array_equal(r["x"], xr) and np.array_equal(r["u"], ur)
    assert r["dt_chem_min"] == np.min(tc)
    assert np.all(r["Gamma"] == 0.0)


def test_zero_step_converges_at_once():
    shape = (2, 3, 4)
    nH, rho, x0, u0 = _medium(shape, 2)
    cp = C.default_params(alpha=_const(1.0), k_ci=_const(0.1))
    rp = RC.default_rt_params(sigma=[3.0], dalpha=_const(0.4))
    r = RC.step(shape, 1.0, nH, rho, x0, u0, 0.0, rp, cp, max_iter=10)
    assert r["iterations"] == 1 and r["converged"]
    # (x_HI goes through n_HI = x n_H and back: one rounding)
    assert np.allclose(r["x"], x0, rtol=4e-16, atol=0) and np.array_equal(r["u"], u0)


def test_fields_give_the_on_the_spot_term():
    """With g_b c_b = 1 the source-function part of Gamma, g S n_HI, is the
    recombination rate to the ground state dalpha n_e n_HII (eq gamma_diff,
    second term); kappa = sigma n_HI with n_HI floored at x_floor n_H."""
    cp = C.default_params(T_per_u=1e3)
    da = np.linspace(0.1, 0.7, 61)
    rp = RC.default_rt_params(nbins=2, sigma=[2.0, 0.5], src_coef=[4.0, 0.25], dalpha=da, x_floor=1e-4)
    nH = np.array([1.0, 2.5, 0.7, 0.0])
    x = np.array([0.3, 1e-6, 1.0, 0.5])
    u = np.array([10.0, 300.0, 1e3, 1.0])
    kappa, S = RC.fields(nH, x, u, rp, cp)
    for i in range(3):
        ne = nH[i] * (1 - x[i])
        nHI = nH[i] * max(x[i], 1e-4)
        T = C.temperature(u[i], 1 - x[i], cp)
        rec = C.interp(da, cp["logT_min"], cp["dlogT"], T) * ne * ne
        for b in range(2):
            assert (1.0 / rp["src_coef"][b]) * S[b, i] * nHI == pytest.approx(rec, rel=1e-13, abs=1e-300)
            assert kappa[b, i] == pytest.approx(rp["sigma"][b] * nHI, rel=1e-15)
    assert np.all(kappa[:, 3] == 0) and np.all(S[:, 3] == 0)          # empty cell
    assert np.all(S[:, 2] == 0)                                       # neutral: no recombinations


@pytest.mark.parametrize("a,da,k", [(1.0, 0.4, 0.25), (2.0, 1.5, 1.0)])
def test_thick_interior_reaches_the_case_b_balance(a, da, k):
    """Uniform medium, constant alpha_A = a, dalpha, k_ci = k, no heating or
    cooling, optically thick cells (kappa h = 200 sigma-units): in the
    central cell J_in vanishes and J = S, the recombination photons are
    re-absorbed on the spot, and after a long step x_HI is the root of
    (alpha_A - dalpha) n_HII = k_ci n_HI, i.e. alpha_B / (alpha_B + k_ci)
    (to the iteration tolerance), not the case-A value alpha_A / (alpha_A + k)."""
    shape = (5, 5, 5)
    n = 125
    nH = np.full(n, 1.0)
    x0 = np.full(n, 0.9)
    u0 = np.full(n, 100.0)
    cp = C.default_params(alpha=_const(a), k_ci=_const(k))
    rp = RC.default_rt_params(sigma=[400.0], dalpha=_const(da))
    r = RC.step(shape, 1.0, nH, nH, x0, u0, 400.0 / a, rp, cp, max_iter=200)
    assert r["converged"]
    xb = (a - da) / (a - da + k)
    xa = a / (a + k)
    c = 62                                                            # centre cell
    assert abs(r["x"][c] - xb) <= 3e-3 * max(xb, 1 - xb), (r["x"][c], xb, xa, r["iterations"])
    assert abs(r["x"][c] - xa) > 10 * 3e-3 * max(xa, 1 - xa)


def test_heating_reaches_the_energy_equation():
    """Fixed species (no reactions, gamma_w = 0) and constant tables: the
    sweep's Heat of the start state, with both weights, heats every cell by
    exactly dt Heat n_HI / rho (Appendix C with H fixed), and the second
    iteration repeats the first."""
    shape = (3, 3, 4)
    nH, rho, x0, u0 = _medium(shape, 4)
    cp = C.default_params()
    rp = RC.default_rt_params(sigma=[1.5], dalpha=_const(0.3), gamma_w=[0.0], heat_in=[2.0],
                              heat_src=[0.7])
    r = RC.step(shape, 1.0, nH, rho, x0, u0, 0.8, rp, cp, max_iter=10)
    from oracle import oracle as O
    kappa, S = RC.fields(nH, x0, u0, rp, cp)
    out = O.sweep(kappa.reshape(1, *shape), S.reshape(1, *shape), 1, gamma_w=[0.0], heat_in=[2.0],
                  heat_src=[0.7])
    H = out["Heat"].reshape(-1)
    assert np.all(H > 0)
    assert r["iterations"] == 2 and r["converged"]
    np.testing.assert_allclose(r["u"], u0 + 0.8 * H * x0 * nH / rho, rtol=1e-13)
    assert np.allclose(r["x"], x0, rtol=4e-16, atol=0)


def test_point_source_in_a_thin_column_reaches_photoionisation_equilibrium():
    """One source at the centre of the first cell of a thin 160-cell column,
    no diffuse emission (dalpha = 0), constant alpha, no collisions: far from
    the source the photon-conserving rate per HI atom is sigma Q / (4 pi r^2)
    (Sect. 2.3), so after a long step x_HI solves alpha n_H (1 - x)^2 =
    Gamma x there (to the shell rate's 2e-4 and the iteration tolerance)."""
    N, a, sig = 160, 1.0, 1e-9
    shape = (N, 1, 1)
    nH = np.full(N, 1.0)
    Q = 4.0 * np.pi * 60.0 ** 2 / sig                     # Gamma = 1 at r = 60
    cp = C.default_params(alpha=_const(a))
    rp = RC.default_rt_params(sigma=[sig], src_pos=[[0.5, 0.5, 0.5]], src_Q=[[Q]])
    r = RC.step(shape, 1.0, nH, nH, np.full(N, 0.5), np.full(N, 100.0), 200.0, rp, cp, max_iter=20)
    assert r["converged"]
    for k in (30, 60, 150):
        G = sig * Q / (4.0 * np.pi * k ** 2)
        x_eq = ((2 * a + G) - np.sqrt((2 * a + G) ** 2 - 4 * a * a)) / (2 * a)
        assert abs(r["x"][k] - x_eq) <= 3e-3 * max(x_eq, 1 - x_eq), (k, r["x"][k], x_eq)
        assert abs(r["Gamma"][k] / G - 1) <= 3e-3


def test_advance_follows_photoionisation_in_time():
    """R4 against the time dependence: a thin column (no recombination, no
    diffuse emission) under one source, advanced to t_end = 2 in radiative
    steps of F = 4 chemical timesteps, follows x_HI(t) = x0 e^{-Gamma t}
    with Gamma = sigma Q / (4 pi r^2) at the chemistry's first-order accuracy:
    the error falls about tenfold when the timestep factors eps_e, eps_HI
    (which set both the sub-steps and, through dt_chem, the radiative steps)
    are ten times smaller; the steps add up to t_end exactly, and the first
    is F times the chemical timestep of the start state."""
    N, sig = 80, 1e-9
    Q = 4.0 * np.pi * 30.0 ** 2 / sig                     # Gamma = 1 at r = 30
    rp = RC.default_rt_params(sigma=[sig], src_pos=[[0.5, 0.5, 0.5]], src_Q=[[Q]])
    nH = np.ones(N)
    exact = 0.9 * math.exp(-1.0 * 2.0)
    errs = []
    for scale in (1.0, 0.1):
        cp = C.default_params()
        cp.update(eps_e=0.2 * scale, eps_HI=0.002 * scale)
        r = RC.advance((N, 1, 1), 1.0, nH, nH, np.full(N, 0.9), np.full(N, 100.0), 2.0, 4.0, rp, cp,
                       max_iter=20, max_steps=100000)
        assert r["t"] == 2.0 and abs(sum(r["dts"]) - 2.0) <= 1e-12 and r["unconverged"] == 0
        errs.append(abs(r["x"][30] - exact) / exact)
    assert errs[0] < 0.3 and 5.0 < errs[0] / errs[1] < 15.0, errs
    cp = C.default_params()
    r1 = RC.step((N, 1, 1), 1.0, nH, nH, np.full(N, 0.9), np.full(N, 100.0), 0.0, rp, cp, 20)
    r = RC.advance((N, 1, 1), 1.0, nH, nH, np.full(N, 0.9), np.full(N, 100.0), 2.0, 4.0, rp, cp, 20, 1)
    assert r["steps"] == 1 and r["dts"][0] == min(4.0 * r1["dt_chem_min"], 2.0)


def test_converged_state_is_a_fixed_point():
    """One more iteration from a converged state moves n_e and u by no more
    than the tolerance (the iteration contracts)."""
    shape = (4, 3, 5)
    nH, rho, x0, u0 = _medium(shape, 3)
    T = np.linspace(1.0, 9.0, 61)
    cp = C.default_params(alpha=2.0 * (10 ** T / 1e4) ** -0.7, k_ci=0.5 * np.exp(-10 ** (5.2 - T)),
                          cool_II=1e-4 * (10 ** T / 1e4) ** 0.5, T_per_u=10.0)
    rp = RC.default_rt_params(sigma=[2.0], dalpha=0.4 * 2.0 * (10 ** T / 1e4) ** -0.7,
                              heat_in=[0.5], heat_src=[0.5], nside=2)
    r = RC.step(shape, 1.0, nH, rho, x0, u0, 0.5, rp, cp, max_iter=100)
    assert r["converged"] and r["iterations"] >= 2
    kappa, S = RC.fields(nH, r["x"], r["u"], rp, cp)
    from oracle import oracle as O
    out = O.sweep(kappa.reshape(1, *shape), S.reshape(1, *shape), 2, gamma_w=rp["gamma_w"],
                  heat_in=rp["heat_in"], heat_src=rp["heat_src"])
    x1, u1, _, _ = C.step(nH, rho, out["Gamma"].reshape(-1), out["Heat"].reshape(-1), x0, u0, 0.5, cp)
    ne0, ne1 = nH * (1 - r["x"]), nH * (1 - x1)
    assert np.all(np.abs(ne1 - ne0) <= cp["eps"] * ne1)
    assert np.all(np.abs(u1 - r["u"]) <= cp["eps"] * u1)
    assert math.isfinite(r["dt_chem_min"]) and r["dt_chem_min"] > 0
