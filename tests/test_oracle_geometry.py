"""Pins of the oracle's ray geometry (Sect. 2.2 parallel rays, Sect. 3.1 ray
grouping) against brute-force cell-by-cell clipping on tiny meshes."""
import itertools

import numpy as np
import pytest

import bruteforce as BF

SHAPES = [(5, 3, 4), (3, 3, 3), (2, 4, 3), (3, 2, 5)]   # (nz, ny, nx)


@pytest.mark.parametrize("shape,nside", [(SHAPES[0], 1), (SHAPES[1], 2), (SHAPES[2], 2),
                                         (SHAPES[3], 4)])
def test_segments_match_bruteforce_chords(oracle_mod, shape, nside):
    O = oracle_mod
    dirs = O.directions(nside)
    nz, ny, nx = shape
    for d, n in enumerate(dirs):
        rays = BF.lattice_rays(n, shape)
        jlo, jhi, klo, khi = O.lattice(shape, nside, d)
        for (j, k) in rays:
            assert jlo <= j <= jhi and klo <= k <= khi, "lattice range misses a ray"
            chords, w = BF.ray_chords(n, shape, j, k)
            cell, dl, s0 = O.ray_segments(shape, nside, d, j, k)
            assert [c for c, _, _ in chords] == cell.tolist()
            np.testing.assert_allclose(dl, [(b - a) / w for _, a, b in chords], atol=1e-12)
            np.testing.assert_allclose(s0, [a for _, a, _ in chords], atol=1e-12)
        # the oracle's lattice range has no ray with a chord that brute force missed
        found = set(rays)
        for j in range(jlo, jhi + 1):
            for k in range(klo, khi + 1):
                if (j, k) not in found:
                    assert len(O.ray_segments(shape, nside, d, j, k)[0]) == 0


@pytest.mark.parametrize("shape,nside", [(SHAPES[0], 2), (SHAPES[3], 4), ((4, 4, 4), 4)])
def test_path_length_invariant_and_grouping(oracle_mod, shape, nside):
    """Every cell gets total path length 1/|n_a| from every direction (the rays
    tile the cell's cross-section), and no cell is crossed twice by rays of the
    same 2x2 group (Sect. 3.1)."""
    O = oracle_mod
    nz, ny, nx = shape
    for d, n in enumerate(O.directions(nside)):
        a, b, c, sig, w, tb, tc = BF.dominant(n)
        total = np.zeros(nx * ny * nz)
        per_group = np.zeros((4, nx * ny * nz), dtype=int)
        for (j, k) in BF.lattice_rays(n, shape):
            chords, _ = BF.ray_chords(n, shape, j, k)
            for cc, s_in, s_out in chords:
                total[cc] += (s_out - s_in) / w
                per_group[(j % 2) + 2 * (k % 2), cc] += 1
        np.testing.assert_allclose(total, 1.0 / w, rtol=1e-12)
        assert per_group.max() == 1


def test_invariant_reported_by_oracle(oracle_mod):
    rng = np.random.default_rng(1)
    k = rng.uniform(0.1, 1.0, (1, 5, 3, 4))
    r = oracle_mod.sweep_raw(k, k, 4)
    assert r["inv_err"] < 1e-12
    assert r["max_hits"] == 1


def test_segment_count_law(oracle_mod):
    """Segments per direction approach N_cells (1 + |t_b| + |t_c|) (Sect. 2.2:
    cost ~ N_m N_d): each slab adds one segment per plane crossing.  Directions
    whose b- and c-crossings coincide (|t_b| = |t_c|) lose segments, so the
    ratio is below 1 and rises towards 1 as such directions become rare."""
    O = oracle_mod
    shape = (12, 12, 12)
    k = np.ones((1,) + shape)
    ratios = []
    for nside in (1, 2, 4, 8):
        r = O.sweep_raw(k, k, nside)
        expect = 0.0
        for d in range(O.ndirs(nside)):
            g = O.dir_geom(nside, d)
            expect += 12 ** 3 * (1 + abs(g["tb"]) + abs(g["tc"]))
        ratios.append(r["nseg"] / expect)
    assert all(x <= 1.0 for x in ratios)
    assert all(b > a for a, b in zip(ratios, ratios[1:]))
    assert ratios[-1] > 0.98
