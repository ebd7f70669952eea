"""Autotuner (art_autotune): it picks a launch shape the mesh can run, the
sweep with that shape still matches the oracle, the persistent cache is
reused, and candidates beyond the local-memory limit are skipped."""
import pytest

from gpu_common import compare_all, oracle_sweep
from paper_1410_0763_amd import media

pytestmark = pytest.mark.gpu


def test_autotune_parity_and_cache(tmp_path):
    print("\n== case autotune ragged 17x23x19, 3 bins, nside 2", flush=True)
    import torch
    from paper_1410_0763_amd import art
    m = media.clumpy_medium((19, 23, 17), nside=2, sigma_ln=1.0, seed=5, nbins=3, name="ragged")
    nb, nz, ny, nx = m.kappa.shape
    cache = str(tmp_path / "tune.json")
    with art.Mesh(nx, ny, nz) as mesh:
        mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
        mesh.set_heating(m.heat_in, m.heat_src)
        r1 = mesh.autotune(m.nside, cache_path=cache)
        print(r1, flush=True)
        assert not r1["cached"] and r1["sweep_ms"] > 0
        assert mesh.get_tuning() == r1["tuning"]
        out = mesh.sweep(m.nside, gamma_w=m.gamma_w, exit_sum=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        compare_all(m, g, oracle_sweep(m))
        r2 = mesh.autotune(m.nside, cache_path=cache)
        assert r2["cached"] and r2["tuning"] == r1["tuning"]
        # a candidate beyond the local-memory limit is skipped
        big = dict(depth=256, subsets=1, waves=1, interleave=4)
        ok = dict(depth=6, subsets=1, waves=1, interleave=2)
        r3 = mesh.autotune(m.nside, candidates=[big, ok])
        assert r3["tuning"] == ok
        with pytest.raises(art.ArtError):
            mesh.autotune(m.nside, candidates=[big])
        assert mesh.get_tuning() == ok      # unchanged by the failed call
