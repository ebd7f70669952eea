"""Pins of the oracle's per-cell form (the sums of eq averaged_intensity at
chosen cells, found by marching only the rays that cross each cell): brute
force on tiny meshes, and the full oracle sweep on ragged multi-bin media."""
import numpy as np
import pytest

import bruteforce as BF
from paper_1410_0763_amd import media


def test_cells_match_brute_force(oracle_mod):
    """Random kappa, S, I_bc: RK4 integration of the transfer equation along
    independently constructed ray chords gives the same J_in and J_exact."""
    O = oracle_mod
    rng = np.random.default_rng(12)
    shape = (3, 4, 5)
    k = rng.uniform(0.05, 2.0, shape)
    s = rng.uniform(0.0, 1.0, shape)
    dirs = O.directions(1)
    J_in, J_ex, _ = BF.bf_sweep(k, s, dirs, I_bc=0.3, method="rk4", nsub=128)
    idx = np.arange(k.size)
    c = O.cells(k[None], s[None], 1, idx, I_bc=0.3)
    np.testing.assert_allclose(c["J_in"][0], J_in.ravel(), rtol=2e-8)
    np.testing.assert_allclose(c["J_exact"][0], J_ex.ravel(), rtol=2e-8)


@pytest.mark.parametrize("shape,nside,nbins", [((11, 17, 13), 2, 3), ((7, 5, 9), 4, 2),
                                               ((1, 6, 1), 2, 1)])
def test_cells_match_full_sweep(oracle_mod, shape, nside, nbins):
    O = oracle_mod
    m = media.clumpy_medium(shape, nside=nside, sigma_ln=1.0, seed=7, nbins=nbins, name="c")
    m.kappa[0, 0, 0, 0] = 0.0            # a vacuum cell (reading Q3)
    full = O.sweep(m.kappa, m.S, nside, gamma_w=m.gamma_w, I_bc=0.2)
    idx = np.arange(m.kappa[0].size)
    c = O.cells(m.kappa, m.S, nside, idx, gamma_w=m.gamma_w, I_bc=0.2)
    for key in ("J_in", "J", "J_exact"):
        np.testing.assert_allclose(c[key], full[key].reshape(nbins, -1), rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(c["Gamma"], full["Gamma"].ravel(), rtol=1e-13)


def test_cells_direction_range_and_order(oracle_mod):
    """Direction sub-ranges add up; the order of the requested cells is free."""
    O = oracle_mod
    m = media.clumpy_medium((9, 8, 10), nside=2, sigma_ln=0.8, seed=9, nbins=2, name="c")
    rng = np.random.default_rng(1)
    idx = rng.permutation(m.kappa[0].size)[:40]
    a = O.cells(m.kappa, m.S, 2, idx, d_range=(0, 17))
    b = O.cells(m.kappa, m.S, 2, idx, d_range=(17, 48))
    full = O.sweep_raw(m.kappa, m.S, 2)
    np.testing.assert_allclose(a["jin_sum"] + b["jin_sum"],
                               full["jin_sum"].reshape(2, -1)[:, idx], rtol=1e-13)
    np.testing.assert_allclose(a["ex_sum"] + b["ex_sum"],
                               full["ex_sum"].reshape(2, -1)[:, idx], rtol=1e-13)
    r = O.cells(m.kappa, m.S, 2, idx[::-1], d_range=(0, 17))
    np.testing.assert_array_equal(r["jin_sum"], a["jin_sum"][:, ::-1])


def test_cells_reject_bad_indices(oracle_mod):
    O = oracle_mod
    k = np.ones((1, 2, 2, 2))
    with pytest.raises(RuntimeError):
        O.cells(k, k, 1, [8])
    with pytest.raises(RuntimeError):
        O.cells(k, k, 1, [-1])
