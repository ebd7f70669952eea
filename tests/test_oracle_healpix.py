"""Pins of the oracle's direction set (Sect. 2.3: HEALPix, 12 Nside^2 equal-area
directions) against published values and properties of the pixelisation."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_nside1_matches_published_base_pixels(oracle_mod):
    z_phi = np.loadtxt(os.path.join(HERE, "golden", "healpix_nside1.txt"))
    n = oracle_mod.directions(1)
    assert n.shape == (12, 3)
    z = z_phi[:, 0]
    phi = z_phi[:, 1] * np.pi
    st = np.sqrt(1 - z * z)
    ref = np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)
    ref[np.abs(ref) < 1e-12] = 0.0
    np.testing.assert_allclose(n, ref, atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 16])
def test_count_norm_and_rings(oracle_mod, nside):
    n = oracle_mod.directions(nside)
    assert n.shape == (12 * nside * nside, 3)
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-15)
    # iso-latitude rings: 4i pixels in the polar caps, 4 Nside in the belt
    zs, counts = np.unique(np.round(n[:, 2], 12), return_counts=True)
    assert len(zs) == 4 * nside - 1
    expect = sorted([4 * i for i in range(1, nside)] * 2 + [4 * nside] * (2 * nside + 1))
    assert sorted(counts.tolist()) == expect
    # the pixels of a ring are equally spaced in azimuth
    for zv in zs:
        ring = n[np.abs(n[:, 2] - zv) < 1e-12]
        phi = np.sort(np.mod(np.arctan2(ring[:, 1], ring[:, 0]), 2 * np.pi))
        gaps = np.diff(np.concatenate([phi, [phi[0] + 2 * np.pi]]))
        np.testing.assert_allclose(gaps, 2 * np.pi / len(ring), atol=1e-12)


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_symmetries_and_balance(oracle_mod, nside):
    n = oracle_mod.directions(nside)
    # antipodal-symmetric set: sum of directions vanishes
    np.testing.assert_allclose(n.sum(axis=0), 0.0, atol=1e-12)
    key = lambda a: set(map(tuple, np.round(a, 10) + 0.0))
    base = key(n)
    for m in (np.diag([-1, 1, 1]), np.diag([1, -1, 1]), np.diag([1, 1, -1]),
              np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])):
        assert key(n @ m.T) == base


def test_equal_area_quadrature(oracle_mod):
    """Equal-area pixels make the centres a quadrature of the sphere: the mean
    of z^2 tends to 1/3 and the error falls like 1/Nside^2."""
    errs = []
    for nside in (2, 4, 8, 16):
        z = oracle_mod.directions(nside)[:, 2]
        errs.append(abs(np.mean(z * z) - 1.0 / 3.0))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 3.0
    assert errs[-1] < 1e-3
