"""Pins of the oracle's transfer arithmetic (Sect. 2.2, eqs rt,
path_averaged_intensity, averaged_intensity, mean_intensity) against closed
forms, numerical integration of the transfer equation and exact identities."""
import numpy as np
import pytest

import bruteforce as BF

SHAPE = (3, 4, 5)   # (nz, ny, nx)


def _run(O, kappa, S, nside, I_bc=0.0, gamma_w=None, h=1.0):
    k = np.asarray(kappa, np.float64)
    s = np.asarray(S, np.float64)
    if k.ndim == 3:
        k, s = k[None], s[None]
    return O.sweep(k, s, nside, gamma_w=gamma_w, h=h, I_bc=I_bc)


def test_vacuum_is_dark(oracle_mod):
    z = np.zeros((1,) + SHAPE)
    r = _run(oracle_mod, z, z, 2)
    for key in ("J_in", "J", "J_exact", "Gamma", "exit_sum"):
        assert np.all(r[key] == 0.0)


def test_free_streaming_keeps_boundary_intensity(oracle_mod):
    """kappa = 0 (reading Q3, phi(0) = 1): nothing is absorbed or emitted."""
    z = np.zeros((1,) + SHAPE)
    r = _run(oracle_mod, z, z, 2, I_bc=1.0)
    np.testing.assert_allclose(r["J_in"], 1.0, atol=1e-14)
    np.testing.assert_allclose(r["exit_sum"], 0.0, atol=1e-12)


@pytest.mark.parametrize("nside,kap", [(1, 0.7), (2, 0.3), (2, 2.5)])
def test_pure_absorber_matches_analytic(oracle_mod, nside, kap):
    """S = 0, I_bc = 1: I = exp(-kappa l) (eq on_the_spot); path averages by quadrature."""
    O = oracle_mod
    k = np.full(SHAPE, kap)
    z = np.zeros(SHAPE)
    r = _run(O, k, z, nside, I_bc=1.0)
    dirs = O.directions(nside)
    J_in, J_ex, exits = BF.bf_sweep(k, z, dirs, I_bc=1.0, method="uniform")
    np.testing.assert_allclose(r["J_in"][0], J_in, rtol=1e-12)
    np.testing.assert_allclose(r["J_exact"][0], J_ex, rtol=1e-12)
    np.testing.assert_allclose(r["exit_sum"][:, 0], exits, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("nside,kap,src", [(1, 0.4, 1.0), (2, 1.3, 0.6)])
def test_uniform_emitter_matches_analytic(oracle_mod, nside, kap, src):
    """I_bc = 0, uniform kappa and S: I = S (1 - exp(-kappa l)); J_exact is its
    angle average, J = J_in + S (eq mean_intensity)."""
    O = oracle_mod
    k = np.full(SHAPE, kap)
    s = np.full(SHAPE, src)
    r = _run(O, k, s, nside)
    dirs = O.directions(nside)
    J_in, J_ex, exits = BF.bf_sweep(k, s, dirs, method="uniform")
    np.testing.assert_allclose(r["J_in"][0], J_in, rtol=1e-12)
    np.testing.assert_allclose(r["J_exact"][0], J_ex, rtol=1e-12)
    np.testing.assert_allclose(r["J"][0], J_in + src, rtol=1e-12)


def test_thick_limit(oracle_mod):
    """Optically thick: J_exact = S in cells one cell or more from every face;
    J_in -> S <phi> = O(1/kappa), so J = J_in + S -> S."""
    O = oracle_mod
    shape = (4, 5, 6)
    kap = 200.0
    k = np.full(shape, kap)
    s = np.full(shape, 0.8)
    r = _run(O, k, s, 2)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(r["J_exact"][0][inner], 0.8, rtol=1e-13)
    assert np.all(r["J_in"][0] * kap <= 0.8 * 60.0)
    assert np.all(r["J_exact"][0] <= 0.8 + 1e-12)


@pytest.mark.parametrize("nside", [1])
def test_random_medium_matches_numerical_integration(oracle_mod, nside):
    """Random kappa, S and I_bc: the segment recursion and the weighted averages
    agree with RK4 integration of dI/dl = kappa (S - I) and Simpson averages."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    k = rng.uniform(0.05, 2.0, SHAPE)
    k[0, 1, 2] = 0.0                          # a vacuum cell (reading Q3)
    s = rng.uniform(0.0, 1.0, SHAPE)
    r = _run(O, k, s, nside, I_bc=0.3)
    dirs = O.directions(nside)
    J_in, J_ex, exits = BF.bf_sweep(k, s, dirs, I_bc=0.3, method="rk4", nsub=64)
    np.testing.assert_allclose(r["J_in"][0], J_in, rtol=2e-8)
    np.testing.assert_allclose(r["J_exact"][0], J_ex, rtol=2e-8)
    np.testing.assert_allclose(r["exit_sum"][:, 0], exits, rtol=2e-8, atol=1e-10)


def test_linearity_in_sources_and_boundary(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    shape = (5, 4, 6)
    k = rng.uniform(0.05, 2.0, (1,) + shape)
    s1, s2 = rng.uniform(0, 1, (2, 1) + shape)
    a = O.sweep(k, s1, 2, I_bc=0.5)
    b = O.sweep(k, s2, 2, I_bc=0.2)
    c = O.sweep(k, 2.0 * s1 - 3.0 * s2, 2, I_bc=2.0 * 0.5 - 3.0 * 0.2)
    for key in ("J_in", "J_exact"):
        np.testing.assert_allclose(c[key], 2.0 * a[key] - 3.0 * b[key], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("nside", [1, 2])
def test_mirror_symmetry(oracle_mod, nside):
    """The direction set and the upstream-face lattice are mirror-symmetric, so
    reflecting the medium reflects the result."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    shape = (5, 4, 6)
    k = rng.uniform(0.05, 2.0, (1,) + shape)
    s = rng.uniform(0, 1, (1,) + shape)
    base = O.sweep(k, s, nside)
    for ax in (1, 2, 3):
        m = O.sweep(np.flip(k, ax), np.flip(s, ax), nside)
        for key in ("J_in", "J_exact"):
            np.testing.assert_allclose(m[key], np.flip(base[key], ax), rtol=1e-10)


def test_axis_swap_symmetry_without_ties(oracle_mod):
    """Nside = 1 has no dominant-axis ties, so swapping x and y commutes with the sweep."""
    O = oracle_mod
    rng = np.random.default_rng(9)
    shape = (4, 5, 5)
    k = rng.uniform(0.05, 2.0, (1,) + shape)
    s = rng.uniform(0, 1, (1,) + shape)
    base = O.sweep(k, s, 1)
    sw = O.sweep(np.swapaxes(k, 2, 3).copy(), np.swapaxes(s, 2, 3).copy(), 1)
    np.testing.assert_allclose(sw["J_in"], np.swapaxes(base["J_in"], 2, 3), rtol=1e-10)


@pytest.mark.parametrize("nside,I_bc,h", [(1, 0.0, 1.0), (2, 0.4, 0.5), (4, 0.0, 2.0)])
def test_photon_balance(oracle_mod, nside, I_bc, h):
    """Exact telescoping identity: h sum_c kappa_c (S_c - J_exact,c) equals
    (1/N_d) sum_d |n_a| sum_rays (I_exit - I_bc)."""
    O = oracle_mod
    rng = np.random.default_rng(11)
    shape = (6, 5, 7)
    k = rng.uniform(0.0, 3.0, (2,) + shape)
    s = rng.uniform(0, 1, (2,) + shape)
    r = O.sweep(k, s, nside, h=h, I_bc=I_bc)
    w = np.array([O.dir_geom(nside, d)["w"] for d in range(O.ndirs(nside))])
    for b in range(2):
        lhs = h * np.sum(k[b] * (s[b] - r["J_exact"][b]))
        rhs = np.sum(w * r["exit_sum"][:, b]) / O.ndirs(nside)
        assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def test_bins_are_independent_and_gamma_affine(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(13)
    shape = (4, 4, 5)
    k = rng.uniform(0.05, 2.0, (3,) + shape)
    s = rng.uniform(0, 1, (3,) + shape)
    g = np.array([1.0, 0.5, 0.25])
    r = O.sweep(k, s, 2, gamma_w=g)
    for b in range(3):
        rb = O.sweep(k[b:b + 1], s[b:b + 1], 2)
        np.testing.assert_allclose(r["J_in"][b], rb["J_in"][0], rtol=1e-14)
    np.testing.assert_allclose(r["Gamma"], np.einsum("b,bzyx->zyx", g, r["J_in"] + s),
                               rtol=1e-14)


def test_direction_ranges_add_up(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(17)
    shape = (5, 6, 4)
    k = rng.uniform(0.05, 2.0, (1,) + shape)
    s = rng.uniform(0, 1, (1,) + shape)
    full = O.sweep_raw(k, s, 2)
    parts = [O.sweep_raw(k, s, 2, d_range=(a, b)) for a, b in ((0, 13), (13, 30), (30, 48))]
    np.testing.assert_allclose(sum(p["jin_sum"] for p in parts), full["jin_sum"], rtol=1e-13)
    np.testing.assert_allclose(sum(p["ex_sum"] for p in parts), full["ex_sum"], rtol=1e-13)
