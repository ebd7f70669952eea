"""Chemistry and energy update (art_chem_step; Appendices B-D) against the
FP64 oracle (oracle/chem.py): every cell of a mixed set of states (neutral,
ionised, hot, cold, empty, fixed species), element by element; and a
128^3 step on the rates of a real sweep, checked at sampled cells and for
the bounds that hold everywhere."""
import numpy as np
import pytest

from oracle import chem as C

pytestmark = pytest.mark.gpu

# Synthetic rate tables on log10 T in [1, 9] (code units; the paper's fits
# are cited, not printed): recombination falling as T^-0.7, collisional
# ionisation and excitation switching on above ~1e5, bremsstrahlung-like
# cooling growing as T^0.5.
LT0, LT1, NT = 1.0, 9.0, 81


def _tables():
    T = 10.0 ** np.linspace(LT0, LT1, NT)
    return dict(alpha=2.0 * (T / 1e4) ** -0.7, k_ci=0.5 * np.exp(-1.6e5 / T),
                cool_I=3e-2 * np.exp(-1.2e5 / T), cool_II=1e-4 * (T / 1e4) ** 0.5)


def _params(T_per_u, max_sub=100000):
    tb = _tables()
    p = C.default_params(nT=NT, logT_min=LT0, logT_max=LT1, **tb)
    p.update(T_per_u=T_per_u, max_sub=max_sub)
    return p, tb


def _states(rng, n):
    nH = rng.lognormal(0.0, 1.0, n)
    rho = nH * rng.uniform(0.9, 1.1, n)
    G = rng.uniform(0.0, 2.0, n) * (rng.uniform(size=n) < 0.8)          # some cells unlit
    H = G * rng.uniform(0.5, 5.0, n)
    x = rng.uniform(0.0, 1.0, n)
    u = 10.0 ** rng.uniform(1.5, 4.5, n)
    # edge cases: empty cells, fully neutral, fully ionised, no radiation at all
    nH[:3] = 0.0
    x[3:6] = 1.0
    x[6:9] = 0.0
    G[9:12] = 0.0
    H[9:12] = 0.0
    return nH, rho, G.astype(np.float32), H.astype(np.float32), x, u


def _run_gpu(nH, rho, G, H, x, u, dt, tb, T_per_u, max_sub=100000):
    import torch
    from paper_1410_0763_amd import art
    d = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(t).cuda()
    tables = {k: d(v) for k, v in tb.items()}
    xg, ug = d(x), d(u)
    dtc = torch.empty(len(nH), dtype=torch.float64, device="cuda")
    ns = torch.empty(len(nH), dtype=torch.int32, device="cuda")
    art.chem_step(d(nH), d(rho), d(G, torch.float32), d(H, torch.float32), xg, ug, dt, tables,
                  LT0, (LT1 - LT0) / (NT - 1), T_per_u=T_per_u, max_sub=max_sub, dt_chem=dtc, nsub=ns)
    torch.cuda.synchronize()
    return xg.cpu().numpy(), ug.cpu().numpy(), dtc.cpu().numpy(), ns.cpu().numpy()


def _rel(a, b):
    scale = np.maximum(np.abs(b), 1e-300)
    return np.abs(a - b) / scale


@pytest.mark.parametrize("dt,max_sub", [(0.3, 100000), (5.0, 100000), (5.0, 3)])
def test_chem_step_matches_oracle_every_cell(dt, max_sub):
    print(f"\n== case chem step dt {dt} max_sub {max_sub}, 600 cells", flush=True)
    rng = np.random.default_rng(int(dt * 10) + max_sub)
    T_per_u = 10.0
    p, tb = _params(T_per_u, max_sub)
    nH, rho, G, H, x, u = _states(rng, 600)
    xr, ur, tr, nr = C.step(nH, rho, G.astype(np.float64), H.astype(np.float64), x, u, dt, p)
    xg, ug, tg, ng = _run_gpu(nH, rho, G, H, x, u, dt, tb, T_per_u, max_sub)
    ex, eu = _rel(xg, xr), _rel(ug, ur)
    fin = np.isfinite(tr)
    # dt_chem divides by the net rate alpha n_e^2 - (k n_e + Gamma) n_HI, which
    # cancels near equilibrium: its error is judged relative to the condition
    # number (sum of the rate's terms over their difference) at the end state
    cond = np.ones(len(nH))
    for i in np.nonzero(fin)[0]:
        nHI = xr[i] * nH[i]
        ne = nH[i] - nHI
        T = C.temperature(ur[i], ne / nH[i], p)
        a = C.interp(p["alpha"], p["logT_min"], p["dlogT"], T)
        k = C.interp(p["k_ci"], p["logT_min"], p["dlogT"], T)
        net = abs(a * ne * ne - (k * ne + float(G[i])) * nHI)
        cond[i] = (a * ne * ne + (k * ne + float(G[i])) * nHI) / net
    et = _rel(tg[fin], tr[fin]) / cond[fin]
    print(f"x_HI max rel {ex.max():.2e}, u max rel {eu.max():.2e}, dt_chem max rel / condition "
          f"{et.max():.2e} (condition up to {cond.max():.1e}), sub-steps {nr.min()}..{nr.max()} "
          f"(equal in {np.mean(ng == nr) * 100:.1f}% of cells)", flush=True)
    assert np.all(ng == nr)
    assert np.array_equal(np.isinf(tg), np.isinf(tr))
    assert ex.max() <= 1e-10 and eu.max() <= 1e-10 and et.max() <= 1e-10
    # empty cells untouched
    assert np.array_equal(xg[:3], x[:3]) and np.array_equal(ug[:3], u[:3]) and np.all(ng[:3] == 0)


def test_chem_step_on_swept_rates_128():
    """The rates of a 128^3 sweep (Gamma and Heat outputs) drive one step of
    every cell; sampled cells against the oracle, bounds everywhere."""
    print("\n== case chem step on the rates of a 128^3 sweep", flush=True)
    import torch
    from paper_1410_0763_amd import art, media
    m = media.clumpy_medium((128, 128, 128), nside=2, sigma_ln=1.5, seed=5100, spheres=16, name="chem128")
    nb, nz, ny, nx = m.kappa.shape
    with art.Mesh(nx, ny, nz) as mesh:
        mesh.set_fields(torch.from_numpy(m.kappa).cuda(), torch.from_numpy(m.S).cuda())
        mesh.set_heating([1.5], [0.1])
        out = mesh.sweep(m.nside)
        G = out["Gamma"].reshape(-1).contiguous()
        H = out["Heat"].reshape(-1).contiguous()
        torch.cuda.synchronize()
    n = nx * ny * nz
    nH = m.density.reshape(-1).astype(np.float64)
    x0 = m.x_hi.reshape(-1).astype(np.float64)
    u0 = np.full(n, 300.0)
    T_per_u = 10.0
    p, tb = _params(T_per_u)
    d = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(t).cuda()
    tables = {k: d(v) for k, v in tb.items()}
    xg, ug = d(x0), d(u0)
    dtc = torch.empty(n, dtype=torch.float64, device="cuda")
    ns = torch.empty(n, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nHd = d(nH)
    e0.record()
    art.chem_step(nHd, nHd, G, H, xg, ug, 0.5, tables, LT0, (LT1 - LT0) / (NT - 1), T_per_u=T_per_u,
                  dt_chem=dtc, nsub=ns)
    e1.record()
    torch.cuda.synchronize()
    xs, us, ts, nss = xg.cpu().numpy(), ug.cpu().numpy(), dtc.cpu().numpy(), ns.cpu().numpy()
    print(f"128^3 step: {e0.elapsed_time(e1):.2f} ms, sub-steps {nss.min()}..{nss.max()} "
          f"(mean {nss.mean():.1f})", flush=True)
    assert np.all((xs >= 0) & (xs <= 1)) and np.all(us >= 10.0 ** LT0 / T_per_u) and np.all(ts > 0)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, n - 1, int(np.argmax(G.cpu().numpy()))], rng.integers(0, n, 40)]))
    Gc, Hc = G.cpu().numpy().astype(np.float64), H.cpu().numpy().astype(np.float64)
    xr, ur, tr, nr = C.step(nH[idx], nH[idx], Gc[idx], Hc[idx], x0[idx], u0[idx], 0.5, p)
    ex, eu = _rel(xs[idx], xr), _rel(us[idx], ur)
    print(f"sampled {len(idx)} cells: x_HI max rel {ex.max():.2e}, u max rel {eu.max():.2e}", flush=True)
    assert np.all(nss[idx] == nr)
    assert ex.max() <= 1e-10 and eu.max() <= 1e-10
