"""Point-source rates (art_point_sources, Sect. 2.3 and Appendix A) against
the oracle: every cell of small ragged meshes (sources at random positions,
at a cell centre, on box corners, faces and cell edges), more sources than
one launch takes, the degenerate calls, and sampled cells of the 128^3
workload the benchmark times."""
import numpy as np
import pytest

from gpu_common import check
from paper_1410_0763_amd import media

pytestmark = pytest.mark.gpu


def _run(kappa, n_abs, pos, Q, e, h=1.0, segs=False):
    import torch
    from paper_1410_0763_amd import art
    nb, nz, ny, nx = kappa.shape
    mesh = art.Mesh(nx, ny, nz, h)
    mesh.set_fields(torch.from_numpy(np.ascontiguousarray(kappa, np.float32)).cuda(),
                    torch.zeros(kappa.shape, dtype=torch.float32).cuda())
    out = mesh.point_sources(pos, Q, torch.from_numpy(np.ascontiguousarray(n_abs, np.float32)).cuda(),
                             e=e, segs=segs)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    mesh.close()
    return res


def _edge_sources(shape, rng, n):
    nz, ny, nx = shape
    pts = [rng.uniform(0, [nx, ny, nz]) for _ in range(n)]
    pts += [[1.5, 2.5, 0.5],            # a cell centre
            [0.0, 0.0, 0.0],            # a box corner
            [nx, ny, nz],               # the opposite corner
            [nx / 2.0, 3.0, 2.0],       # cell edges inside the box
            [0.0, ny / 3.0, nz - 0.25]]  # a face
    return np.array(pts, dtype=np.float64)


@pytest.mark.parametrize("shape,nb,h", [((13, 11, 17), 3, 1.0), ((8, 21, 6), 1, 0.6),
                                        ((16, 16, 16), 4, 1.0)])
def test_every_cell_small(shape, nb, h):
    from oracle import oracle as O
    print(f"\n== case point sources {shape} nb={nb} h={h}", flush=True)
    rng = np.random.default_rng(sum(shape) + nb)
    kappa = rng.uniform(0.0, 1.5, (nb,) + shape).astype(np.float32)
    kappa[:, 2, 3, :] = 0.0                                   # a vacuum row
    n_abs = rng.uniform(0.2, 2.0, shape).astype(np.float32)
    n_abs[1, 1, 1] = 0.0                                      # no absorbers
    pos = _edge_sources(shape, rng, 3)
    Q = rng.uniform(0.1, 3.0, (len(pos), nb))
    e = rng.uniform(0.0, 2.0, nb)
    got = _run(kappa, n_abs, pos, Q, e, h=h, segs=True)
    ref = O.point(kappa, n_abs, pos, Q, e, h=h)
    check(f"point {shape}:Gamma", got["Gamma"].ravel(), ref["Gamma"])
    check(f"point {shape}:Heat", got["Heat"].ravel(), ref["Heat"])
    assert got["Gamma"][1, 1, 1] == 0.0
    assert np.all(got["segs"] >= len(pos))


def test_more_sources_than_one_launch():
    """70 sources: two launches, the second adding to the first."""
    from oracle import oracle as O
    print("\n== case point sources, 70 sources", flush=True)
    rng = np.random.default_rng(70)
    shape = (6, 5, 9)
    kappa = rng.uniform(0.05, 1.0, (2,) + shape).astype(np.float32)
    n_abs = rng.uniform(0.5, 1.5, shape).astype(np.float32)
    pos = rng.uniform(0, [9, 5, 6], size=(70, 3))
    Q = rng.uniform(0.1, 1.0, (70, 2))
    e = np.array([0.5, 1.0])
    got = _run(kappa, n_abs, pos, Q, e, segs=True)
    ref = O.point(kappa, n_abs, pos, Q, e)
    check("point 70 sources:Gamma", got["Gamma"].ravel(), ref["Gamma"])
    check("point 70 sources:Heat", got["Heat"].ravel(), ref["Heat"])
    assert np.all(got["segs"] >= 70)


def test_degenerate_calls_and_errors():
    """No sources (zeros), no energies (Heat 0), a source on its own cell's
    centre alone in a 1-cell mesh, and the argument errors."""
    import torch
    from paper_1410_0763_amd import art
    print("\n== case point sources, degenerate calls", flush=True)
    kappa = np.full((1, 3, 4, 5), 0.4, np.float32)
    n_abs = np.ones((3, 4, 5), np.float32)
    z = _run(kappa, n_abs, np.zeros((0, 3)), np.zeros((0, 1)), None)
    assert np.all(z["Gamma"] == 0.0) and np.all(z["Heat"] == 0.0)
    g = _run(kappa, n_abs, [[2.5, 1.5, 0.5]], [[1.0]], None)
    assert np.all(g["Heat"] == 0.0) and np.all(g["Gamma"] > 0.0)
    one = _run(np.full((1, 1, 1, 1), 0.8, np.float32), np.ones((1, 1, 1), np.float32),
               [[0.5, 0.5, 0.5]], [[1.0]], None)
    want = (1.0 - np.exp(-0.4)) / (4.0 * np.pi / 3.0 * 0.125)
    assert one["Gamma"][0, 0, 0] == pytest.approx(want, rel=1e-6)
    mesh = art.Mesh(5, 4, 3, 1.0)
    mesh.set_fields(torch.from_numpy(kappa).cuda(), torch.zeros(kappa.shape).cuda())
    nab = torch.from_numpy(n_abs).cuda()
    for pos, Q, e in (([[5.5, 1.0, 1.0]], [[1.0]], None), ([[1.0, -0.1, 1.0]], [[1.0]], None),
                      ([[1.0, 1.0, np.nan]], [[1.0]], None), ([[1.0, 1.0, 1.0]], [[-1.0]], None),
                      ([[1.0, 1.0, 1.0]], [[np.inf]], None), ([[1.0, 1.0, 1.0]], [[1.0]], [np.nan])):
        with pytest.raises(art.ArtError) as ei:
            mesh.point_sources(pos, Q, nab, e=e)
        assert ei.value.code == -1
    mesh.close()


def test_workload_128_sampled_cells():
    """The 128^3 workload with 16 sources and 4 bins, as the benchmark runs it,
    at sampled cells (corners, the sources' own cells, the most opaque cells,
    random cells)."""
    import os
    from oracle import oracle as O
    print("\n== case point sources 128^3, 16 sources, sampled cells", flush=True)
    w = media.point_sources()
    m = w.medium
    nb, nz, ny, nx = m.kappa.shape
    got = _run(m.kappa, w.n_abs, w.pos, w.Q, w.e)
    rng = np.random.default_rng(128)
    pts = {(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, 0), (nz - 1, 0, nx - 1)}
    for p in w.pos:
        pts.add((min(int(p[2]), nz - 1), min(int(p[1]), ny - 1), min(int(p[0]), nx - 1)))
    for f in np.argsort(m.kappa[0].ravel())[-6:]:
        pts.add(tuple(int(v) for v in np.unravel_index(f, (nz, ny, nx))))
    while len(pts) < 70:
        pts.add(tuple(int(rng.integers(0, s)) for s in (nz, ny, nx)))
    idx = np.array(sorted((z * ny + y) * nx + x for z, y, x in pts), dtype=np.int64)
    ref = O.point(m.kappa, w.n_abs, w.pos, w.Q, w.e, cell_idx=idx,
                  nthreads=min(16, os.cpu_count() or 1))
    assert np.all(np.isfinite(got["Gamma"])) and np.all(got["Gamma"] >= 0.0)
    check("point 128 sampled:Gamma", got["Gamma"].ravel()[idx], ref["Gamma"])
    check("point 128 sampled:Heat", got["Heat"].ravel()[idx], ref["Heat"])


def test_new_fields_rebuild_the_pack():
    """The kappa pack follows art_set_fields: new values and a new bin count
    (1 -> 3 -> 2) each give the oracle's rates for the fields then loaded."""
    import torch
    from oracle import oracle as O
    from paper_1410_0763_amd import art
    print("\n== case point sources after new fields", flush=True)
    rng = np.random.default_rng(99)
    shape = (7, 9, 8)
    mesh = art.Mesh(shape[2], shape[1], shape[0], 1.0)
    n_abs = rng.uniform(0.5, 1.5, shape).astype(np.float32)
    nab = torch.from_numpy(n_abs).cuda()
    pos = np.array([[1.2, 7.7, 3.3], [6.5, 0.4, 6.9]])
    for nb in (1, 3, 2):
        kappa = rng.uniform(0.05, 1.2, (nb,) + shape).astype(np.float32)
        mesh.set_fields(torch.from_numpy(kappa).cuda(), torch.zeros(kappa.shape).cuda())
        Q = rng.uniform(0.5, 1.5, (2, nb))
        e = rng.uniform(0.1, 1.0, nb)
        out = mesh.point_sources(pos, Q, nab, e=e)
        torch.cuda.synchronize()
        ref = O.point(kappa, n_abs, pos, Q, e)
        check(f"point new fields nb={nb}:Gamma", out["Gamma"].cpu().numpy().ravel(), ref["Gamma"])
        check(f"point new fields nb={nb}:Heat", out["Heat"].cpu().numpy().ravel(), ref["Heat"])
    mesh.close()
