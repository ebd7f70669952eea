"""Pins of the oracle's point-source rates (Sect. 2.3 and the photon-conserving
form of Appendix A) against what geometry and the transfer equation fix:
closed forms in uniform media (with the line's entry and exit found by a
different method than the oracle's), photon conservation along a column, the
optically thin flux formula, brute-force line integrals of kappa, and scaling
and linearity properties."""
import numpy as np
import pytest

from oracle import oracle as O

FOUR_PI_3 = 4.0 * np.pi / 3.0


def _face_hits(p, c):
    """Entry and exit distances of the line from p through the centre of cell
    c, found by intersecting the line with the six face planes and keeping the
    hits that lie on the face squares (not the slab method)."""
    p = np.asarray(p, float)
    q = np.asarray(c, float) + 0.5
    d = q - p
    L = np.linalg.norm(d)
    u = d / L if L > 0 else np.array([1.0, 0.0, 0.0])
    ts = []
    for ax in range(3):
        if u[ax] == 0.0:
            continue
        for plane in (c[ax], c[ax] + 1.0):
            t = (plane - p[ax]) / u[ax]
            x = p + t * u
            o = [a for a in range(3) if a != ax]
            if all(c[a] - 1e-12 <= x[a] <= c[a] + 1 + 1e-12 for a in o):
                ts.append(t)
    ts = sorted(ts)
    t_in, t_out = ts[0], ts[-1]
    return max(t_in, 0.0), t_out


def _sources(shape, rng, n):
    nz, ny, nx = shape
    pts = [rng.uniform(0, [nx, ny, nz]) for _ in range(n)]
    pts.append(np.array([1.5, 0.5, 2.5]))          # at a cell centre
    pts.append(np.array([0.0, 0.0, 0.0]))          # on a box corner
    pts.append(np.array([nx, 2.0, 1.0]))           # on a face, on cell edges
    return np.array(pts)


def test_uniform_medium_closed_form():
    """tau = kappa h r_in and the rate of each (source, cell) pair in closed
    form, at every cell of a ragged box, several bins and sources."""
    rng = np.random.default_rng(7)
    shape = (5, 4, 6)
    nz, ny, nx = shape
    h = 0.7
    kb = np.array([0.2, 1.3, 0.01])
    kappa = np.broadcast_to(kb[:, None, None, None], (3,) + shape).copy()
    n = 2.5
    pos = _sources(shape, rng, 4)
    Q = rng.uniform(0.5, 2.0, (len(pos), 3))
    e = np.array([0.3, 1.0, 2.0])
    want_g = np.zeros(nx * ny * nz)
    want_h = np.zeros(nx * ny * nz)
    for cid in range(nx * ny * nz):
        c = (cid % nx, (cid // nx) % ny, cid // (nx * ny))
        for s, p in enumerate(pos):
            rin, rout = _face_hits(p, c)
            pair = O.point_pair(kappa, p, cid, h=h)
            assert pair["r_in"] == pytest.approx(rin, abs=1e-9)
            assert pair["r_out"] == pytest.approx(rout, abs=1e-9)
            np.testing.assert_allclose(pair["tau"], kb * h * rin, rtol=1e-12, atol=1e-13)
            vol = FOUR_PI_3 * h ** 3 * (rout ** 3 - rin ** 3)
            ab = Q[s] * np.exp(-kb * h * rin) * (1.0 - np.exp(-kb * h * (rout - rin)))
            want_g[cid] += ab.sum() / (n * vol)
            want_h[cid] += (ab * e).sum() / (n * vol)
    r = O.point(kappa, np.full(shape, n), pos, Q, e, h=h)
    np.testing.assert_allclose(r["Gamma"], want_g, rtol=1e-10)
    np.testing.assert_allclose(r["Heat"], want_h, rtol=1e-10)


def test_photon_conservation_along_a_column():
    """On a 1 x 1 x N column lit from the centre of its bottom face the shells
    of successive cells are adjacent, so the photons they absorb add up to
    Q (1 - e^{-tau_total}) (Appendix A)."""
    rng = np.random.default_rng(3)
    N = 40
    h = 1.3
    kappa = rng.uniform(0.0, 0.6, (2, N, 1, 1))
    nab = rng.uniform(0.5, 3.0, (N, 1, 1))
    Q = np.array([[2.0, 5.0]])
    tot = np.zeros(2)
    for b in range(2):
        Qb = np.zeros((1, 2))
        Qb[0, b] = Q[0, b]
        g = O.point(kappa, nab, [[0.5, 0.5, 0.0]], Qb, h=h)["Gamma"]
        k = np.arange(N)
        vol = FOUR_PI_3 * h ** 3 * ((k + 1.0) ** 3 - k ** 3.0)
        tot[b] = np.sum(g * nab.ravel() * vol)
    want = Q[0] * (1.0 - np.exp(-kappa.reshape(2, -1).sum(axis=1) * h))
    np.testing.assert_allclose(tot, want, rtol=1e-12)


def test_optically_thin_limit_is_the_flux_formula():
    """Far from the source in a thin medium the rate per absorber approaches
    sigma Q / (4 pi r^2) (the flux f = L e^{-tau} / (4 pi r^2) of Sect. 2.3
    with sigma = kappa / n)."""
    N = 400
    kappa = np.full((1, N, 1, 1), 1e-9)
    nab = np.full((N, 1, 1), 2.0)
    g = O.point(kappa, nab, [[0.5, 0.5, 0.5]], [[3.0]])["Gamma"]
    r = np.arange(N) * 1.0                       # distance to the cell centres
    sigma = 1e-9 / 2.0
    for k in (50, 150, 399):
        assert g[k] / (sigma * 3.0 / (4 * np.pi * r[k] ** 2)) == pytest.approx(1.0, abs=2e-4)


def test_tau_equals_brute_force_line_integral():
    """tau of random media against a midpoint-rule integral of kappa along the
    line (10^6 samples), for random sources and cells."""
    rng = np.random.default_rng(11)
    shape = (6, 7, 5)
    nz, ny, nx = shape
    kappa = rng.uniform(0.05, 2.0, (1,) + shape)
    for _ in range(25):
        p = rng.uniform(0, [nx, ny, nz])
        cid = int(rng.integers(0, nx * ny * nz))
        c = np.array([cid % nx, (cid // nx) % ny, cid // (nx * ny)])
        pair = O.point_pair(kappa, p, cid)
        q = c + 0.5
        u = (q - p) / np.linalg.norm(q - p)
        M = 1_000_000
        t = (np.arange(M) + 0.5) * (pair["r_in"] / M)
        x = p[None, :] + t[:, None] * u[None, :]
        ijk = np.clip(np.floor(x).astype(int), 0, [nx - 1, ny - 1, nz - 1])
        brute = kappa[0, ijk[:, 2], ijk[:, 1], ijk[:, 0]].sum() * (pair["r_in"] / M)
        assert pair["tau"][0] == pytest.approx(brute, rel=2e-4, abs=1e-6)
        assert pair["dtau"][0] == pytest.approx(kappa[0, c[2], c[1], c[0]] *
                                                (pair["r_out"] - pair["r_in"]), rel=1e-12)


def test_source_at_the_target_centre():
    """p at the centre of its own cell: the shell is the ball of radius 1/2
    (reading P2: the line runs along +x)."""
    kappa = np.full((1, 3, 3, 3), 0.8)
    cid = 13
    g = O.point(kappa, np.ones((3, 3, 3)), [[1.5, 1.5, 1.5]], [[1.0]], cell_idx=[cid])["Gamma"]
    want = (1.0 - np.exp(-0.8 * 0.5)) / (FOUR_PI_3 * 0.5 ** 3)
    assert g[0] == pytest.approx(want, rel=1e-13)


def test_scaling_linearity_and_empty_cells():
    rng = np.random.default_rng(5)
    shape = (4, 5, 3)
    kappa = rng.uniform(0.1, 1.0, (2,) + shape)
    nab = rng.uniform(0.5, 2.0, shape)
    nab[1, 2, 1] = 0.0
    pos = _sources(shape, rng, 2)
    Q = rng.uniform(0.5, 2.0, (len(pos), 2))
    e = np.array([0.5, 1.5])
    base = O.point(kappa, nab, pos, Q, e)
    # cell size: kappa / s and n / s^3 with h = s leave every optical depth and
    # absorber count, hence every rate, unchanged
    s = 2.0
    scaled = O.point(kappa / s, nab / s ** 3, pos, Q, e, h=s)
    np.testing.assert_allclose(scaled["Gamma"], base["Gamma"], rtol=1e-12)
    # bins and sources add
    parts = np.zeros_like(base["Heat"])
    for i in range(len(pos)):
        for b in range(2):
            Qi = np.zeros_like(Q)
            Qi[i, b] = Q[i, b]
            parts += O.point(kappa, nab, pos, Qi, e)["Heat"]
    np.testing.assert_allclose(parts, base["Heat"], rtol=1e-12)
    # a cell without absorbers has no rate
    flat = (1 * shape[1] + 2) * shape[2] + 1
    assert base["Gamma"][flat] == 0.0 and base["Heat"][flat] == 0.0
    # sampled cells equal the whole-mesh result
    idx = np.array([0, 7, 59, 33])
    sub = O.point(kappa, nab, pos, Q, e, cell_idx=idx)
    np.testing.assert_allclose(sub["Gamma"], base["Gamma"][idx], rtol=1e-15)


def test_bad_arguments_are_rejected():
    kappa = np.ones((1, 2, 2, 2))
    with pytest.raises(ValueError):
        O.point(kappa, np.ones((2, 2, 2)), [[2.5, 0.5, 0.5]], [[1.0]])
    with pytest.raises(ValueError):
        O.point(kappa, np.ones((2, 2, 2)), [[0.5, 0.5, 0.5]], [[1.0]], cell_idx=[8])
    with pytest.raises(ValueError):
        O.point_pair(kappa, [0.5, -0.1, 0.5], 0)
