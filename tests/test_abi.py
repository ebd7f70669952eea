"""The C-ABI library loads and exports every entry point include/art.h
declares; host-only argument checks (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="art.h"):
    with open(os.path.join(ROOT, "include", header)) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(art_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared() == sorted(art.EXPORTS)


def test_nn_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared("art_nn.h") == sorted(art.NN_EXPORTS)


def test_surrogate_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared("art_surrogate.h") == sorted(art.SG_EXPORTS)


def test_point_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared("art_point.h") == sorted(art.PT_EXPORTS)


def test_diag_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared("art_diag.h") == sorted(art.DIAG_EXPORTS)
    L = art.load()
    ns = (ctypes.c_float * 5)()
    assert L.art_diag_release_cost(0, 16, ns) == -1 and L.art_diag_release_cost(4, 16, None) == -1


def test_chem_header_and_binding_agree():
    from paper_1410_0763_amd import art
    assert _declared("art_chem.h") == sorted(art.CHEM_EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1410_0763_amd import art
    L = art.load()
    for name in (_declared() + _declared("art_nn.h") + _declared("art_surrogate.h") +
                 _declared("art_point.h") + _declared("art_chem.h") + _declared("art_diag.h")):
        assert hasattr(L, name), name


def test_chem_argument_checks_without_gpu():
    """Bad sizes, pointers and parameters are rejected before any launch."""
    from paper_1410_0763_amd import art
    L = art.load()
    p = ctypes.c_void_p(1)
    good = dict(nT=61, logT_min=1.0, dlogT=0.1, alpha=p, k_ci=p, cool_I=p, cool_II=p, T_per_u=1.0,
                eps=1e-3, eps_e=0.2, eps_HI=0.002, max_iter=100, max_sub=1000)

    def call(n=4, dt=1.0, nullcell=False, **kw):
        prm = art.ChemParams(**dict(good, **kw))
        cell = None if nullcell else p
        return L.art_chem_step(n, cell, p, p, p, p, p, dt, ctypes.byref(prm), None, None, None)
    assert call(n=0) == 0
    assert call(n=-1) == -1
    assert call(nullcell=True) == -1
    assert call(dt=-1.0) == -1 and call(dt=float("inf")) == -1
    assert call(nT=1) == -1 and call(dlogT=0.0) == -1 and call(alpha=None) == -1
    assert call(T_per_u=0.0) == -1 and call(eps=0.0) == -1 and call(eps_e=0.0, eps_HI=0.0) == -1
    assert call(max_iter=0) == -1 and call(max_sub=-1) == -1
    assert L.art_chem_step(4, p, p, p, p, p, p, 1.0, None, None, None, None) == -1


def test_rt_chem_argument_checks_without_gpu():
    """The coupled step rejects bad parameters and a short workspace before any
    device work; the workspace size follows the mesh and the bin count."""
    import numpy as np
    from paper_1410_0763_amd import art
    L = art.load()
    p = ctypes.c_void_p(1)
    h = ctypes.c_void_p()
    assert L.art_create_mesh(4, 5, 6, 1.0, ctypes.byref(h)) == 0
    w1, w2 = L.art_rt_chem_workspace(h, 1), L.art_rt_chem_workspace(h, 2)
    assert w1 > 120 * (8 * 5 + 4 * 4) and w2 - w1 >= 2 * 120 * 4
    assert L.art_rt_chem_workspace(h, 0) == -1 and L.art_rt_chem_workspace(None, 1) == -1
    cp = art.ChemParams(61, 1.0, 0.1, p, p, p, p, 1.0, 1e-3, 0.2, 0.002, 100, 1000)
    one = (ctypes.c_float * 1)(1.0)
    neg = (ctypes.c_float * 1)(-1.0)
    res = art.RtChemResult()

    def call(nb=1, sig=one, dal=p, nside=1, xf=1e-6, mi=10, dt=1.0, wb=w1, cpp=cp, ns=0):
        rp = art.RtChemParams(nb, ctypes.cast(sig, ctypes.c_void_p), ctypes.cast(one, ctypes.c_void_p), dal,
                              None, None, None, nside, xf, mi, ns, None, None, None)
        return L.art_rt_chem_step(h, ctypes.byref(rp), ctypes.byref(cpp), p, p, p, p, dt, p, wb, None, None,
                                  ctypes.byref(res), None)
    assert call(nb=0) == -1 and call(nb=5) == -1
    assert call(sig=neg) == -1 and call(dal=None) == -1 and call(nside=0) == -1
    assert call(xf=0.0) == -1 and call(xf=1.5) == -1 and call(mi=0) == -1
    assert call(ns=-1) == -1 and call(ns=2) == -1                    # sources without positions
    assert call(dt=-1.0) == -1 and call(dt=float("nan")) == -1
    assert call(wb=w1 - 1) == -1 and b"workspace" in L.art_last_error()
    assert call(cpp=art.ChemParams(1, 1.0, 0.1, p, p, p, p, 1.0, 1e-3, 0.2, 0.002, 100, 1000)) == -1
    run = art.RtChemRun()

    def adv(nb=1, t_end=1.0, F=1.0, ms=10, out=run):
        rp = art.RtChemParams(nb, ctypes.cast(one, ctypes.c_void_p), ctypes.cast(one, ctypes.c_void_p), p,
                              None, None, None, 1, 1e-6, 10, 0, None, None, None)
        return L.art_rt_chem_advance(h, ctypes.byref(rp), ctypes.byref(cp), p, p, p, p, t_end, F, ms, p, w1,
                                     None, None, None if out is None else ctypes.byref(out), None)
    assert adv(t_end=-1.0) == -1 and adv(t_end=float("inf")) == -1 and adv(t_end=float("nan")) == -1
    assert adv(F=0.0) == -1 and adv(F=float("inf")) == -1 and adv(ms=0) == -1 and adv(out=None) == -1
    assert adv(nb=0) == -1 and b"nbins" in L.art_last_error()          # the step's own checks come first
    assert L.art_destroy_mesh(h) == 0


def test_point_argument_checks_without_gpu():
    """Sources outside the box, negative or non-finite photon rates and calls
    before set_fields are rejected before any device work."""
    import numpy as np
    from paper_1410_0763_amd import art
    L = art.load()
    dp = ctypes.POINTER(ctypes.c_double)
    p = ctypes.c_void_p(1)
    assert L.art_point_sources(None, 1, None, None, None, p, p, None, None, None) == -1
    h = ctypes.c_void_p()
    assert L.art_create_mesh(4, 5, 6, 1.0, ctypes.byref(h)) == 0
    pos = np.array([[1.0, 1.0, 1.0]])
    Q = np.array([[1.0]])
    args = lambda pp, qq: (pp.ctypes.data_as(dp), qq.ctypes.data_as(dp), None, p, p, None, None, None)
    assert L.art_point_sources(h, 1, *args(pos, Q)) == -4          # no fields yet
    assert b"art_set_fields" in L.art_last_error()
    assert L.art_destroy_mesh(h) == 0


def test_checkpoint_digest_is_sha256():
    """The checkpoint digest against hashlib's SHA-256, across the padding
    boundaries (55, 56, 63, 64 bytes) and several blocks."""
    import hashlib
    import random
    from paper_1410_0763_amd import surrogate as SG
    rnd = random.Random(3)
    for n in (0, 1, 3, 55, 56, 57, 63, 64, 65, 119, 120, 128, 1000, 65537):
        data = bytes(rnd.getrandbits(8) for _ in range(n))
        assert SG.sha256(data) == hashlib.sha256(data).digest(), n


def test_surrogate_argument_checks_without_gpu():
    """Shapes and arguments the surrogate cannot take are rejected before any
    device call."""
    from paper_1410_0763_amd import art
    L = art.load()
    h = ctypes.c_void_p()
    assert L.art_surrogate_create(48, 8, 8, 0, ctypes.byref(h)) == -1          # nx not a multiple of 32
    assert b"multiple of 32" in L.art_last_error()
    assert L.art_surrogate_create(32, 0, 8, 0, ctypes.byref(h)) == -1
    assert L.art_surrogate_create(32, 8, 8, 0, None) == -1
    assert L.art_surrogate_create(320, 320, 320, 0, ctypes.byref(h)) == -5     # above the 2 GiB buffers
    assert L.art_surrogate_n_params(None) == -1
    assert L.art_surrogate_destroy(None) == 0
    assert L.art_sweep_surrogate(None, None, None, None, 2, 16, None, 1.0, None, None, None, None) == -1
    assert L.art_sha256(None, 5, ctypes.create_string_buffer(32)) == -1


def test_nn_argument_checks_without_gpu():
    """Null pointers and bad sizes are rejected before any launch."""
    from paper_1410_0763_amd import art
    L = art.load()
    p = ctypes.c_void_p(1)
    assert L.art_conv3d_fwd(None, 16, p, None, 4, 4, 32, 1, None, p, None, None) == -1
    assert L.art_conv3d_fwd(p, 8, p, None, 4, 4, 32, 1, None, p, None, None) == -1
    assert L.art_conv3d_fwd(p, 16, p, None, 4, 4, 48, 1, None, p, None, None) == -1
    assert b"multiple of 32" in L.art_last_error()
    assert L.art_conv3d_bwd_weight(p, 32, p, 4, 4, 24, p, 1 << 30, p, None, None) == -1
    assert b"multiple of 16" in L.art_last_error()
    need = L.art_conv3d_bwd_weight_workspace(32, 4, 4, 32)
    assert need == 16 * (27 * 32 * 32 + 32)                  # 4 rows x 4 chunks of 1 plane
    assert L.art_conv3d_bwd_weight(p, 32, p, 4, 4, 32, p, need - 1, p, None, None) == -1
    assert b"workspace" in L.art_last_error()
    assert L.art_conv3d_bwd_weight(p, 32, p, 4, 4, 32, None, need, p, None, None) == -1
    assert L.art_conv3d_bwd_weight_workspace(8, 4, 4, 32) == -1
    assert L.art_conv3d_bwd_weight_workspace(32, 4, 4, 40) == -1
    assert L.art_conv3d_bwd_weight_workspace(32, 128, 128, 128) == 256 * (27 * 32 * 32 + 32)
    assert L.art_nn_relu_grad(None, None, 4, p, None) == -1
    assert L.art_nn_prep_weights(p, 20, p, p, None) == -1
    assert L.art_nn_adamw(p, p, p, p, 10, 1e-3, 0.9, 0.999, 1e-8, 0.0, 0, None) == -1


def test_host_only_calls():
    from paper_1410_0763_amd import art
    L = art.load()
    assert L.art_ndirs(8) == 768
    assert L.art_ndirs(0) == -1
    assert b"nside" in L.art_last_error()
    h = ctypes.c_void_p()
    assert L.art_create_mesh(0, 4, 4, 1.0, ctypes.byref(h)) == -1
    assert L.art_create_mesh(4, 4, 4, -1.0, ctypes.byref(h)) == -1
    assert L.art_create_mesh(4, 4, 4, 1.0, None) == -1
    assert L.art_create_mesh(4, 5, 6, 0.5, ctypes.byref(h)) == 0
    t = art.Tuning()
    assert L.art_get_tuning(h, ctypes.byref(t)) == 0
    assert t.depth > 0 and t.subsets > 0 and t.waves > 0
    for bad in (art.Tuning(32, 1, 0, 2), art.Tuning(0, 1, 8, 2), art.Tuning(300, 1, 8, 2),
                art.Tuning(32, 65, 8, 2), art.Tuning(32, 1, 9, 2), art.Tuning(32, 1, 8, 5)):
        assert L.art_set_tuning(h, ctypes.byref(bad)) == -1
    ok = art.Tuning(16, 2, 4, 4)
    assert L.art_set_tuning(h, ctypes.byref(ok)) == 0
    assert L.art_get_tuning(h, ctypes.byref(t)) == 0
    assert (t.depth, t.subsets, t.waves, t.interleave) == (16, 2, 4, 4)
    # heating weights and a sweep before set_fields are state errors, caught
    # before any GPU work
    assert L.art_set_heating(h, None, None) == -4
    assert L.art_set_heating(None, None, None) == -1
    o = art.Outputs()
    assert L.art_sweep(h, 2, None, ctypes.c_float(0.0), ctypes.byref(o), None) == -4
    assert L.art_destroy_mesh(h) == 0
    assert L.art_destroy_mesh(None) == 0


def test_tune_cache_file_round_trip_and_rejections(tmp_path):
    """The autotune cache file (host only): bad files are rejected with the
    cache unchanged, a valid file loads and saves back to the same entries."""
    from paper_1410_0763_amd import art
    art.tune_cache("clear")
    good = tmp_path / "good.txt"
    good.write_text("art-tune-cache 1\n7 8 4 6 1 1 3 101.5\n4 2 1 4 1 1 2 0.75\n")
    bad_magic = tmp_path / "bad1.txt"
    bad_magic.write_text("not-a-cache 1\n")
    bad_entry = tmp_path / "bad2.txt"
    bad_entry.write_text("art-tune-cache 1\n7 8 4 0 1 1 3 1.0\n")       # depth 0
    bad_line = tmp_path / "bad3.txt"
    bad_line.write_text("art-tune-cache 1\n7 8 4 6 1 1\n")
    for p in (bad_magic, bad_entry, bad_line, tmp_path / "missing.txt"):
        with pytest.raises(art.ArtError):
            art.tune_cache("load", p)
    out = tmp_path / "out.txt"
    art.tune_cache("save", out)
    assert out.read_text().splitlines() == ["art-tune-cache 1"]          # still empty
    art.tune_cache("load", good)
    art.tune_cache("save", out)
    lines = sorted(out.read_text().splitlines()[1:])
    assert lines == ["4 2 1 4 1 1 2 0.75", "7 8 4 6 1 1 3 101.5"]
    art.tune_cache("clear")
    with pytest.raises(KeyError):
        art.tune_cache("frobnicate")
    L = art.load()
    assert L.art_tune_cache(7, None) == -1                                 # unknown op
