"""Pins of the oracle's diffuse photo-heating rate (eq heat_diff with its
frequency integrals folded into per-bin weights, reading Q12):
Heat = sum_b heat_in_b J_in_b + heat_src_b S_b."""
import numpy as np
import pytest

SHAPE = (5, 4, 6)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def _medium(nb=2, seed=3):
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.05, 2.0, (nb,) + SHAPE)
    s = rng.uniform(0.0, 1.0, (nb,) + SHAPE)
    return k, s


def test_equal_weights_reduce_to_gamma(O):
    """With heat_in = heat_src = g the heating sum is the rate of eq gamma_diff."""
    k, s = _medium()
    g = np.array([0.7, 0.2])
    r = O.sweep(k, s, 2, gamma_w=g, heat_in=g, heat_src=g)
    np.testing.assert_allclose(r["Heat"], r["Gamma"], rtol=1e-14, atol=0)


def test_no_weights_no_heat_and_linearity(O):
    k, s = _medium()
    r0 = O.sweep(k, s, 1)
    assert not np.any(r0["Heat"])
    a = O.sweep(k, s, 1, heat_in=[1.0, 0.0], heat_src=[0.0, 0.0])["Heat"]
    b = O.sweep(k, s, 1, heat_in=[0.0, 0.0], heat_src=[0.0, 2.0])["Heat"]
    ab = O.sweep(k, s, 1, heat_in=[1.0, 0.0], heat_src=[0.0, 2.0])["Heat"]
    np.testing.assert_allclose(ab, a + b, rtol=1e-14)
    # bin 0's J_in term alone, bin 1's source term alone
    np.testing.assert_allclose(a, r0["J_in"][0], rtol=1e-14)
    np.testing.assert_allclose(b, 2.0 * s[1], rtol=1e-14)


def test_free_streaming_closed_form(O):
    """kappa = 0: every ray keeps I_bc, so J_in = I_bc in every cell and
    Heat = heat_in I_bc + heat_src S exactly (the source does not emit into
    rays of a medium without opacity)."""
    z = np.zeros((1,) + SHAPE)
    s = np.random.default_rng(9).uniform(0.0, 1.0, (1,) + SHAPE)
    r = O.sweep(z, s, 2, I_bc=1.5, heat_in=[0.3], heat_src=[0.25])
    np.testing.assert_allclose(r["Heat"], 0.3 * 1.5 + 0.25 * s[0], rtol=1e-13)


def test_cells_match_full_sweep(O):
    k, s = _medium(nb=3, seed=8)
    k = k.reshape((3,) + SHAPE)
    idx = np.array([0, 7, 33, 119])
    hin, hsrc = [0.1, 0.4, 0.9], [0.05, 0.0, 0.3]
    full = O.sweep(k, s, 2, heat_in=hin, heat_src=hsrc)
    c = O.cells(k, s, 2, idx, heat_in=hin, heat_src=hsrc)
    np.testing.assert_allclose(c["Heat"], full["Heat"].ravel()[idx], rtol=1e-13)
