"""art_point_sources_noalloc (the entry point for callers that cannot
allocate) against art_point_sources through the C-ABI: the same kernels on
the same kappa pack, so the rates must agree bit for bit, on two calls in a
row, the second with a smaller mesh and fewer sources (the static scratch
keeps the first call's pack, which the second must not use)."""
import ctypes

import numpy as np
import pytest

from paper_1410_0763_amd import media

pytestmark = pytest.mark.gpu


def _noalloc(mesh, w, Gamma, Heat, segs):
    import torch
    from paper_1410_0763_amd import art
    L = art.load()
    f = L.art_point_sources_noalloc
    vp = ctypes.c_void_p
    f.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
    f.restype = ctypes.c_int
    pos = np.ascontiguousarray(w.pos, dtype=np.float64)
    Q = np.ascontiguousarray(w.Q, dtype=np.float64)
    e = np.ascontiguousarray(w.e, dtype=np.float64)
    n_abs = torch.from_numpy(np.ascontiguousarray(w.n_abs, dtype=np.float32)).cuda()
    rc = f(mesh._h, len(pos), pos.ctypes.data, Q.ctypes.data, e.ctypes.data, n_abs.data_ptr(),
           Gamma.data_ptr(), Heat.data_ptr(), segs.data_ptr(),
           torch.cuda.current_stream().cuda_stream)
    return rc, n_abs


def _case(shape, nsrc, seed):
    import torch
    from paper_1410_0763_amd import art
    w = media.point_sources(shape=shape, nsrc=nsrc, nbins=4, seed=seed, spheres=4)
    m = w.medium
    nb, nz, ny, nx = m.kappa.shape
    print(f"\n== case noalloc point sources {shape} x {nsrc} sources, {nb} bins", flush=True)
    mesh = art.Mesh(nx, ny, nz, m.cell_size)
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
    ref = mesh.point_sources(w.pos, w.Q, torch.from_numpy(w.n_abs).cuda(), e=w.e, segs=True)
    G = torch.full(m.shape, -1.0, device="cuda")
    H = torch.full(m.shape, -1.0, device="cuda")
    S = torch.zeros(m.shape, dtype=torch.int32, device="cuda")
    rc, _keep = _noalloc(mesh, w, G, H, S)
    assert rc == 0, art.load().art_last_error().decode()
    torch.cuda.synchronize()
    for key, got in (("Gamma", G), ("Heat", H), ("segs", S)):
        a, b = got.cpu().numpy(), ref[key].cpu().numpy()
        print(f"{key}: max |noalloc - plain| {np.max(np.abs(a.astype(np.float64) - b)):.3e}", flush=True)
        assert np.array_equal(a, b), key
    mesh.close()


def test_noalloc_matches_point_sources_twice():
    _case((40, 36, 44), 9, 7100)
    _case((21, 17, 13), 3, 7200)     # smaller mesh, fewer sources: the pack is rebuilt


def test_noalloc_rejects_a_mesh_beyond_the_scratch():
    import torch
    from paper_1410_0763_amd import art
    n = 260                          # 260^3 cells x 4 floats > 16 Mi floats
    mesh = art.Mesh(n, n, n)
    z = torch.zeros((4, n, n, n), device="cuda")
    mesh.set_fields(z + 0.1, z)
    G = torch.empty((n, n, n), device="cuda")
    L = art.load()
    f = L.art_point_sources_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 8
    f.restype = ctypes.c_int
    pos = np.array([[1.0, 2.0, 3.0]])
    Q = np.ones((1, 4))
    rc = f(mesh._h, 1, pos.ctypes.data, Q.ctypes.data, None, G.data_ptr(), G.data_ptr(), None, None,
           torch.cuda.current_stream().cuda_stream)
    assert rc == -5, (rc, L.art_last_error().decode())
    assert "scratch" in L.art_last_error().decode()
    del z
    mesh.close()
    torch.cuda.synchronize()
