"""Failure paths through the C-ABI on the GPU: rejected fields leave a usable
mesh, oversize requests return an error code, and a mesh held by a live batch
refuses whatever would reallocate or re-shape the buffers its graph captured."""
import numpy as np
import pytest

from gpu_common import check, oracle_sweep
from paper_1410_0763_amd import media

pytestmark = pytest.mark.gpu


def _upload(mesh, m):
    import torch
    mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())


def test_invalid_fields_rejected_mesh_still_sweeps():
    """NaN or negative kappa, or non-finite S, give ART_E_INVAL; the mesh keeps
    its previous fields, and the next sweep equals the one before, bitwise,
    and the oracle."""
    import torch
    from paper_1410_0763_amd import art
    m = media.clumpy_medium((14, 11, 9), nside=2, sigma_ln=1.0, seed=91, nbins=2, name="inval")
    print("\n== case invalid fields on", m.shape, flush=True)
    nb, nz, ny, nx = m.kappa.shape
    with art.Mesh(nx, ny, nz) as mesh:
        _upload(mesh, m)
        before = {k: v.cpu().numpy() for k, v in mesh.sweep(m.nside, gamma_w=m.gamma_w).items()}
        bads = []
        k = m.kappa.copy(); k[1, 3, 4, 5] = np.nan; bads.append((k, m.S))
        k = m.kappa.copy(); k[0, 0, 0, 0] = -1e-3; bads.append((k, m.S))
        s = m.S.copy(); s[1, 13, 10, 8] = np.inf; bads.append((m.kappa, s))
        for kk, ss in bads:
            for dev in (True, False):
                kt, stt = torch.from_numpy(np.ascontiguousarray(kk)), torch.from_numpy(np.ascontiguousarray(ss))
                if dev:
                    kt, stt = kt.cuda(), stt.cuda()
                with pytest.raises(art.ArtError) as ei:
                    mesh.set_fields(kt, stt)
                assert ei.value.code == -1, str(ei.value)
        after = {k: v.cpu().numpy() for k, v in mesh.sweep(m.nside, gamma_w=m.gamma_w).items()}
        torch.cuda.synchronize()
    for key in ("J_in", "J", "J_exact", "Gamma"):
        assert np.array_equal(before[key], after[key]), key
    ref = oracle_sweep(m)
    for key in ("J_in", "J", "J_exact", "Gamma"):
        check(f"after rejected fields:{key}", after[key], ref[key])


def test_oversize_requests_return_codes():
    """Requests past the 32-bit offsets of the march and out-of-range sizes
    return error codes (no allocation, no launch)."""
    import torch
    from paper_1410_0763_amd import art
    print("\n== case oversize 4096 x 4096 x 1 at nside 64", flush=True)
    with pytest.raises(art.ArtError) as ei:
        art.Mesh(5000, 4, 4)
    assert ei.value.code == -1
    with art.Mesh(4096, 4096, 1) as mesh:
        z = torch.zeros((1, 1, 4096, 4096), device="cuda")
        mesh.set_fields(z + 0.5, z)
        with pytest.raises(art.ArtError) as ei:
            mesh.sweep(64, out=dict(J_in=torch.empty_like(z)))
        assert ei.value.code == -5, str(ei.value)
        with pytest.raises(art.ArtError) as ei:
            mesh.sweep(65, out=dict(J_in=torch.empty_like(z)))
        assert ei.value.code == -1, str(ei.value)
        del z
    torch.cuda.synchronize()


def test_live_batch_guards_its_meshes():
    """While a batch holds two meshes: re-tuning, autotuning, a new bin count,
    a sweep at a larger Nside and destruction give ART_E_STATE; a plain sweep
    at a smaller Nside and a direction range are allowed and match the oracle;
    the next replay rebuilds the replaced tables and still matches the oracle;
    after the batch is gone the meshes take every call again."""
    import torch
    from paper_1410_0763_amd import art
    meds = [media.clumpy_medium((12, 10, 9), nside=4, sigma_ln=1.0, seed=93, nbins=2, name="g0"),
            media.clumpy_medium((9, 13, 11), nside=2, sigma_ln=1.0, seed=94, nbins=1, name="g1")]
    print("\n== case batch guard", [(m.shape, m.nside, m.nbins) for m in meds], flush=True)
    meshes = []
    for m in meds:
        nb, nz, ny, nx = m.kappa.shape
        mesh = art.Mesh(nx, ny, nz)
        _upload(mesh, m)
        mesh.set_heating(m.heat_in, m.heat_src)
        meshes.append(mesh)
    refs = [oracle_sweep(m) for m in meds]
    batch = art.Batch(meshes, [m.nside for m in meds], [m.gamma_w for m in meds])

    def replay_and_check(tag):
        outs = batch.launch()
        batch.stats()
        for m, o, r in zip(meds, outs, refs):
            for key in ("J_in", "J_exact", "Gamma", "Heat"):
                check(f"{tag}:{m.name}:{key}", o[key].cpu().numpy(), r[key])

    replay_and_check("replay 1")
    m0 = meshes[0]
    refused = [
        lambda: m0.set_tuning(4, 1, 1, 2),
        lambda: m0.autotune(4, candidates=[dict(depth=4, subsets=1, waves=1, interleave=2)]),
        lambda: m0.sweep(8),
        lambda: m0.set_fields(torch.zeros((1,) + meds[0].shape, device="cuda"),
                              torch.zeros((1,) + meds[0].shape, device="cuda")),
        lambda: m0.close(),
    ]
    for i, call in enumerate(refused):
        with pytest.raises(art.ArtError) as ei:
            call()
        assert ei.value.code == -4, f"call {i}: {ei.value}"
    assert m0._h, "a refused destroy keeps the mesh"
    # allowed: a smaller Nside and a direction range (they replace the tables)
    small = media.Medium("g0_nside2", meds[0].kappa, meds[0].S, 2, meds[0].gamma_w,
                         heat_in=meds[0].heat_in, heat_src=meds[0].heat_src)
    got = {k: v.cpu().numpy() for k, v in m0.sweep(2, gamma_w=small.gamma_w).items()}
    ref2 = oracle_sweep(small)
    for key in ("J_in", "J_exact"):
        check(f"plain nside 2 on a batched mesh:{key}", got[key], ref2[key])
    from oracle import oracle as O
    A1, A2 = meshes[1].sweep_range(2, 5, 30)
    rr = O.sweep_raw(meds[1].kappa, meds[1].S, 2, d_range=(5, 30))
    check("range on a batched mesh:A1", A1.cpu().numpy(), rr["jin_sum"])
    replay_and_check("replay after plain sweeps")
    replay_and_check("replay 3")
    batch.close()
    m0.set_tuning(4, 1, 1, 2)
    got = {k: v.cpu().numpy() for k, v in m0.sweep(meds[0].nside, gamma_w=meds[0].gamma_w).items()}
    check("after the batch, re-tuned:J_in", got["J_in"], refs[0]["J_in"])
    for mesh in meshes:
        mesh.close()
    torch.cuda.synchronize()
