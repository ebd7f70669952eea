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


# ---------------------------------------------------------------------------
# Azimuthal phase of the belt rings at Nside >= 2.  The pins above (ring
# sizes, spacing, symmetries, quadrature) hold for either phase of the belt
# rings, so a wrong ring parity would pass them.  Two facts fix the phase.
# ---------------------------------------------------------------------------

def _base_centres():
    z_phi = np.loadtxt(os.path.join(HERE, "golden", "healpix_nside1.txt"))
    st = np.sqrt(1 - z_phi[:, 0] ** 2)
    phi = z_phi[:, 1] * np.pi
    return np.stack([st * np.cos(phi), st * np.sin(phi), z_phi[:, 0]], axis=1)


def _is_centre(n, v):
    return bool(np.min(np.linalg.norm(n - v, axis=1)) < 1e-12)


def _tie_count(n):
    """Directions whose largest |component| is shared by two axes."""
    a = np.abs(n)
    m = a.max(axis=1, keepdims=True)
    return int(np.sum(np.sum(a >= m - 1e-12, axis=1) > 1))


def _ring_set_with_belt_parity(nside, parity):
    """HEALPix RING centres with the belt-ring offset s = parity(i); used to
    show that the pins below reject a wrong parity."""
    N = nside
    out = []
    for i in range(1, 4 * N):
        if i < N or i > 3 * N:
            ip = i if i < N else 4 * N - i
            z = 1 - ip * ip / (3.0 * N * N)
            z = z if i < N else -z
            npix, dphi, phi0 = 4 * ip, np.pi / (2 * ip), np.pi / (4 * ip)
        else:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * N)
            npix, dphi = 4 * N, np.pi / (2 * N)
            phi0 = 0.5 * dphi if parity(i, N) else 0.0
        st = np.sqrt((1 - z) * (1 + z))
        for j in range(npix):
            p = phi0 + dphi * j
            out.append([st * np.cos(p), st * np.sin(p), z])
    n = np.array(out)
    n[np.abs(n) < 1e-12] = 0.0
    return n


def _base_centre_pin(n, nside):
    """Gorski et al. (2005): every base pixel is divided into an Nside x Nside
    grid of equal-area pixels.  The middle of an odd grid is a pixel centre,
    the middle of an even grid a vertex shared by four pixels, so each of the
    12 base-pixel centres is a pixel centre at odd Nside and not at even."""
    return all(_is_centre(n, b) == (nside % 2 == 1) for b in _base_centres())


# dominant-axis ties (reading Q2): 8, 16, 24, 56 directions at Nside 2, 4, 8, 16
TIES = {1: 0, 2: 8, 4: 16, 8: 24, 16: 56}


@pytest.mark.parametrize("nside", [2, 3, 4, 5, 8, 16])
def test_base_pixel_centres_fix_belt_phase(oracle_mod, nside):
    assert _base_centre_pin(oracle_mod.directions(nside), nside)


@pytest.mark.parametrize("nside", sorted(TIES))
def test_dominant_axis_tie_counts(oracle_mod, nside):
    assert _tie_count(oracle_mod.directions(nside)) == TIES[nside]


def test_belt_phase_pins_reject_wrong_parity(oracle_mod):
    """The belt offset is s = (i - Nside + 1) mod 2.  The same construction
    reproduces the oracle exactly; with s = i mod 2 (wrong for even Nside)
    both pins fail at every even Nside."""
    right = lambda i, N: (i - N + 1) % 2
    wrong = lambda i, N: i % 2
    for nside in (2, 4, 8, 16):
        np.testing.assert_allclose(_ring_set_with_belt_parity(nside, right),
                                   oracle_mod.directions(nside), atol=1e-14)
        bad = _ring_set_with_belt_parity(nside, wrong)
        assert not _base_centre_pin(bad, nside)
        assert _tie_count(bad) != TIES[nside]
