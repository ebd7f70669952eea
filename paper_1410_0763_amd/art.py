"""Python binding of libart (include/art.h): argument marshalling only.

Every step of the sweep runs in the HIP library; torch tensors serve as device
buffers and torch streams as HIP streams.  If libart.so is missing or cannot
be loaded, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libart.so")

ART_OK = 0
ERRORS = {-1: "ART_E_INVAL", -2: "ART_E_NOMEM", -3: "ART_E_HIP", -4: "ART_E_STATE",
          -5: "ART_E_UNSUPPORTED"}
MAX_BINS = 4
MAX_NSIDE = 64

# Every symbol include/art.h declares.
EXPORTS = ("art_create_mesh", "art_destroy_mesh", "art_set_fields", "art_sweep",
           "art_sweep_range", "art_sweep_stats", "art_set_tuning", "art_get_tuning",
           "art_batch_create", "art_batch_launch", "art_batch_stats", "art_batch_destroy",
           "art_ndirs", "art_last_error", "art_autotune", "art_set_heating", "art_schedule",
           "art_autotune_class", "art_tune_cache", "art_sweep_batched", "art_graph_launch",
           "art_graph_destroy")
# include/art_nn.h: layers of the learned surrogate
NN_EXPORTS = ("art_conv3d_fwd", "art_conv3d_bwd_weight", "art_conv3d_bwd_weight_workspace",
              "art_nn_relu_grad", "art_nn_prep_weights", "art_nn_mse", "art_nn_adamw",
              "art_nn_features", "art_nn_expand", "art_nn_log_ratio", "art_nn_ood_count",
              "art_nn_sq_weights")
# include/art_surrogate.h: the surrogate object, its gate and checkpoints
SG_EXPORTS = ("art_surrogate_create", "art_surrogate_destroy", "art_surrogate_n_params",
              "art_surrogate_set_stats", "art_surrogate_get_stats", "art_surrogate_fit_stats",
              "art_surrogate_features", "art_surrogate_make_pair", "art_surrogate_gradients",
              "art_surrogate_train_step", "art_surrogate_infer", "art_surrogate_param",
              "art_surrogate_save", "art_surrogate_load", "art_sweep_surrogate", "art_sha256")
# include/art_point.h: rates from point sources
PT_EXPORTS = ("art_point_sources", "art_point_sources_noalloc")
# include/art_chem.h: chemistry and energy update of a radiative step
CHEM_EXPORTS = ("art_chem_step", "art_rt_chem_workspace", "art_rt_chem_step", "art_rt_chem_advance")
# include/art_diag.h: measurements behind design decisions
DIAG_EXPORTS = ("art_diag_release_cost",)


class ArtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


OUTPUT_KEYS = ("J_in", "J", "J_exact", "Gamma", "exit_sum", "Heat")


class Outputs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in OUTPUT_KEYS]

    @classmethod
    def of(cls, out: dict):
        return cls(*(_ptr(out.get(k)) for k in OUTPUT_KEYS))


class ChemParams(ctypes.Structure):
    """art_chem_params (include/art_chem.h); the tables are device pointers."""
    _fields_ = [("nT", ctypes.c_int), ("logT_min", ctypes.c_double), ("dlogT", ctypes.c_double),
                ("alpha", ctypes.c_void_p), ("k_ci", ctypes.c_void_p), ("cool_I", ctypes.c_void_p),
                ("cool_II", ctypes.c_void_p), ("T_per_u", ctypes.c_double), ("eps", ctypes.c_double),
                ("eps_e", ctypes.c_double), ("eps_HI", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("max_sub", ctypes.c_int)]


class RtChemParams(ctypes.Structure):
    """art_rt_chem_params (include/art_chem.h): host per-bin arrays, device dalpha."""
    _fields_ = [("nbins", ctypes.c_int), ("sigma", ctypes.c_void_p), ("src_coef", ctypes.c_void_p),
                ("dalpha", ctypes.c_void_p), ("gamma_w", ctypes.c_void_p), ("heat_in", ctypes.c_void_p),
                ("heat_src", ctypes.c_void_p), ("nside", ctypes.c_int), ("x_floor", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("nsrc", ctypes.c_int), ("src_pos", ctypes.c_void_p),
                ("src_Q", ctypes.c_void_p), ("src_e", ctypes.c_void_p)]


class RtChemResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("dt_chem_min", ctypes.c_double)]


class RtChemRun(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("iterations", ctypes.c_int), ("unconverged", ctypes.c_int),
                ("t", ctypes.c_double), ("dt_chem_min", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("subsets", ctypes.c_int), ("waves", ctypes.c_int),
                ("interleave", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libart.so and declare the C signatures (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libart.so not built at {path}; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, i, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
    L.art_create_mesh.argtypes = [i, i, i, d, ctypes.POINTER(vp)]
    L.art_destroy_mesh.argtypes = [vp]
    L.art_set_fields.argtypes = [vp, i, vp, vp, i, vp]
    L.art_sweep.argtypes = [vp, i, vp, f, ctypes.POINTER(Outputs), vp]
    L.art_sweep_range.argtypes = [vp, i, i, i, f, vp, vp, vp]
    L.art_sweep_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    L.art_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.art_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.art_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i), i, ctypes.POINTER(vp), f,
                                   ctypes.POINTER(Outputs), i, ctypes.POINTER(vp), vp]
    L.art_batch_launch.argtypes = [vp, vp]
    L.art_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_float)]
    L.art_batch_destroy.argtypes = [vp]
    L.art_ndirs.argtypes = [i]
    L.art_set_heating.argtypes = [vp, vp, vp]
    L.art_autotune.argtypes = [vp, i, ctypes.POINTER(Tuning), i, ctypes.POINTER(Tuning),
                               ctypes.POINTER(ctypes.c_float), vp]
    L.art_schedule.argtypes = [i, i, i, ctypes.POINTER(Tuning), vp, ctypes.c_longlong,
                               ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(i)]
    L.art_autotune_class.argtypes = [vp, i, ctypes.POINTER(Tuning), i, ctypes.POINTER(Tuning),
                                     ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i), vp]
    L.art_tune_cache.argtypes = [i, ctypes.c_char_p]
    L.art_sweep_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i), i, ctypes.POINTER(vp),
                                    ctypes.POINTER(Outputs), ctypes.POINTER(vp), vp]
    L.art_graph_launch.argtypes = [vp, vp]
    L.art_graph_destroy.argtypes = [vp]
    L.art_last_error.restype = ctypes.c_char_p
    fp = ctypes.POINTER(ctypes.c_float)
    L.art_conv3d_fwd.argtypes = [vp, i, vp, vp, i, i, i, i, vp, vp, vp, vp]
    L.art_conv3d_bwd_weight.argtypes = [vp, i, vp, i, i, i, vp, ctypes.c_longlong, vp, vp, vp]
    L.art_conv3d_bwd_weight_workspace.argtypes = [i, i, i, i]
    L.art_conv3d_bwd_weight_workspace.restype = ctypes.c_longlong
    L.art_nn_relu_grad.argtypes = [vp, vp, i, vp, vp]
    L.art_nn_prep_weights.argtypes = [vp, i, vp, vp, vp]
    L.art_nn_mse.argtypes = [vp, vp, vp, i, vp, vp, vp, vp]
    L.art_nn_sq_weights.argtypes = [vp, i, f, vp, vp, vp]
    L.art_nn_adamw.argtypes = [vp, vp, vp, vp, i, f, f, f, f, f, i, vp]
    L.art_nn_features.argtypes = [vp, vp, vp, i, fp, fp, vp, vp]
    L.art_nn_expand.argtypes = [vp, vp, i, vp, vp]
    L.art_nn_log_ratio.argtypes = [vp, vp, i, vp, vp]
    L.art_nn_ood_count.argtypes = [vp, i, fp, fp, vp, vp]
    cp, ip = ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)
    L.art_surrogate_create.argtypes = [i, i, i, ctypes.c_ulonglong, ctypes.POINTER(vp)]
    L.art_surrogate_destroy.argtypes = [vp]
    L.art_surrogate_n_params.argtypes = [vp]
    L.art_surrogate_set_stats.argtypes = [vp, fp, fp, fp, fp, f]
    L.art_surrogate_get_stats.argtypes = [vp, fp, fp, fp, fp, fp]
    L.art_surrogate_fit_stats.argtypes = [vp, i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), f, vp]
    L.art_surrogate_features.argtypes = [vp, vp, vp, vp, vp, vp]
    L.art_surrogate_make_pair.argtypes = [vp, vp, i, i, f, vp, vp, vp, vp, vp]
    L.art_surrogate_gradients.argtypes = [vp, vp, vp, vp, vp, vp]
    L.art_surrogate_train_step.argtypes = [vp, vp, vp, vp, f, f, vp, vp]
    L.art_surrogate_infer.argtypes = [vp, vp, vp, vp]
    L.art_surrogate_param.argtypes = [vp, i, i, vp, i, vp]
    L.art_surrogate_save.argtypes = [vp, cp, vp]
    L.art_surrogate_load.argtypes = [vp, cp, vp]
    L.art_sweep_surrogate.argtypes = [vp, vp, vp, vp, i, i, vp, f, ctypes.POINTER(Outputs), ip, fp, vp]
    L.art_sha256.argtypes = [vp, ctypes.c_ulonglong, vp]
    L.art_point_sources.argtypes = [vp, i, vp, vp, vp, vp, vp, vp, vp, vp]
    L.art_point_sources_noalloc.argtypes = [vp, i, vp, vp, vp, vp, vp, vp, vp, vp]
    L.art_chem_step.argtypes = [ctypes.c_longlong, vp, vp, vp, vp, vp, vp, d,
                                ctypes.POINTER(ChemParams), vp, vp, vp]
    L.art_rt_chem_workspace.argtypes = [vp, i]
    L.art_rt_chem_workspace.restype = ctypes.c_longlong
    L.art_rt_chem_step.argtypes = [vp, ctypes.POINTER(RtChemParams), ctypes.POINTER(ChemParams), vp, vp,
                                   vp, vp, d, vp, ctypes.c_longlong, vp, vp, ctypes.POINTER(RtChemResult),
                                   vp]
    L.art_rt_chem_advance.argtypes = [vp, ctypes.POINTER(RtChemParams), ctypes.POINTER(ChemParams), vp, vp,
                                      vp, vp, d, d, i, vp, ctypes.c_longlong, vp, vp,
                                      ctypes.POINTER(RtChemRun), vp]
    L.art_diag_release_cost.argtypes = [i, i, ctypes.POINTER(ctypes.c_float)]
    for name in EXPORTS + NN_EXPORTS + SG_EXPORTS + PT_EXPORTS + CHEM_EXPORTS + DIAG_EXPORTS:
        if name not in ("art_last_error", "art_rt_chem_workspace"):
            getattr(L, name).restype = i
    _lib = L
    return L


def _check(rc):
    if rc != ART_OK:
        raise ArtError(rc, load().art_last_error().decode())
    return rc


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def ndirs(nside: int) -> int:
    return 12 * nside * nside


class Mesh:
    """A mesh of nx*ny*nz cubic cells (library-owned device state)."""

    def __init__(self, nx: int, ny: int, nz: int, cell_size: float = 1.0):
        L = load()
        h = ctypes.c_void_p()
        _check(L.art_create_mesh(nx, ny, nz, float(cell_size), ctypes.byref(h)))
        self._h = h
        self.shape = (nz, ny, nx)
        self.nbins = 0

    def close(self):
        """Free the mesh (ArtError ART_E_STATE, mesh kept, while a live batch holds it)."""
        if getattr(self, "_h", None):
            _check(load().art_destroy_mesh(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- fields ----------------------------------------------------------
    def set_fields(self, kappa, S, stream=None):
        """kappa, S: float32 tensors (nbins, nz, ny, nx), CUDA or CPU."""
        import torch
        assert kappa.shape == S.shape and kappa.dim() == 4 and tuple(kappa.shape[1:]) == self.shape
        kappa = kappa.contiguous()
        S = S.contiguous()
        assert kappa.dtype == torch.float32 and S.dtype == torch.float32
        on_dev = 1 if kappa.is_cuda else 0
        assert S.is_cuda == kappa.is_cuda
        sp = _stream_ptr(stream) if on_dev else ctypes.c_void_p(0)
        _check(load().art_set_fields(self._h, kappa.shape[0], _ptr(kappa), _ptr(S), on_dev, sp))
        self.nbins = kappa.shape[0]

    def set_heating(self, heat_in=None, heat_src=None):
        """Weights of the Heat output (art_set_heating): per bin, of J_in and of S."""
        def arr(v):
            if v is None:
                return None
            a = (ctypes.c_float * self.nbins)(*[float(x) for x in v])
            return ctypes.cast(a, ctypes.c_void_p), a
        hi, hs = arr(heat_in), arr(heat_src)
        _check(load().art_set_heating(self._h, hi[0] if hi else None, hs[0] if hs else None))

    # -- tuning ----------------------------------------------------------
    def set_tuning(self, depth, subsets, waves, interleave=2):
        t = Tuning(depth, subsets, waves, interleave)
        _check(load().art_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().art_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, nside: int, candidates=None, cache_path=None, stream=None) -> dict:
        """Fastest launch shape for this mesh and Nside (art_autotune), set on
        the mesh.  With cache_path, results persist in a JSON file keyed by
        mesh shape, Nside and bins, and a cached entry is reused without
        timing."""
        import json
        key = f"{self.shape[2]}x{self.shape[1]}x{self.shape[0]}|nside{nside}|bins{self.nbins}"
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
            if key in cache:
                t = cache[key]["tuning"]
                self.set_tuning(t["depth"], t["subsets"], t["waves"], t["interleave"])
                return dict(cache[key], cached=True)
        cands, n = None, 0
        if candidates:
            n = len(candidates)
            cands = (Tuning * n)(*[Tuning(c["depth"], c["subsets"], c["waves"], c["interleave"])
                                   for c in candidates])
        best = Tuning()
        ms = ctypes.c_float()
        _check(load().art_autotune(self._h, nside, cands, n, ctypes.byref(best), ctypes.byref(ms),
                                   _stream_ptr(stream)))
        rec = dict(tuning=best.as_dict(), sweep_ms=ms.value)
        if cache_path:
            cache[key] = rec
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        return dict(rec, cached=False)

    def autotune_class(self, nside: int, candidates=None, stream=None) -> dict:
        """art_autotune_class: the launch shape of this mesh's shape class,
        Nside and bins from the library's cache, or timed and cached."""
        cands, n = None, 0
        if candidates:
            n = len(candidates)
            cands = (Tuning * n)(*[Tuning(c["depth"], c["subsets"], c["waves"], c["interleave"])
                                   for c in candidates])
        best = Tuning()
        ms = ctypes.c_float()
        cached = ctypes.c_int()
        _check(load().art_autotune_class(self._h, nside, cands, n, ctypes.byref(best),
                                         ctypes.byref(ms), ctypes.byref(cached), _stream_ptr(stream)))
        return dict(tuning=best.as_dict(), sweep_ms=ms.value, cached=bool(cached.value))

    # -- sweeps ----------------------------------------------------------
    def alloc_outputs(self, nside: int, exit_sum: bool = False, device="cuda"):
        import torch
        nb = self.nbins
        shp = (nb,) + self.shape
        out = dict(J_in=torch.empty(shp, device=device), J=torch.empty(shp, device=device),
                   J_exact=torch.empty(shp, device=device),
                   Gamma=torch.empty(self.shape, device=device),
                   Heat=torch.empty(self.shape, device=device))
        if exit_sum:
            out["exit_sum"] = torch.empty((ndirs(nside), nb), device=device)
        return out

    def sweep(self, nside: int, gamma_w=None, I_bc: float = 0.0, out=None, exit_sum=False,
              stream=None):
        """Full sweep; returns (and fills) a dict of device tensors."""
        if out is None:
            out = self.alloc_outputs(nside, exit_sum)
        o = Outputs.of(out)
        gw = None
        if gamma_w is not None:
            arr = (ctypes.c_float * self.nbins)(*[float(v) for v in gamma_w])
            gw = ctypes.cast(arr, ctypes.c_void_p)
        _check(load().art_sweep(self._h, nside, gw, float(I_bc), ctypes.byref(o),
                                _stream_ptr(stream)))
        return out

    def stats(self) -> dict:
        """Segments marched (per bin) and event times of the last sweep (synchronises)."""
        seg = ctypes.c_longlong()
        mms = ctypes.c_float()
        sms = ctypes.c_float()
        _check(load().art_sweep_stats(self._h, ctypes.byref(seg), ctypes.byref(mms),
                                      ctypes.byref(sms)))
        return dict(segments=seg.value, march_ms=mms.value, sweep_ms=sms.value)

    def point_sources(self, pos, Q, n_abs, e=None, out=None, segs: bool = False, stream=None,
                      noalloc: bool = False):
        """Photon-conserving rates per absorber from point sources
        (art_point_sources, or art_point_sources_noalloc with noalloc=True):
        pos (nsrc, 3) and Q (nsrc, nbins) host arrays, e (nbins,) or None,
        n_abs a device float32 tensor of the mesh's shape.  Returns (and
        fills) a dict Gamma, Heat (and segs) of device tensors."""
        import numpy as np
        import torch
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        nsrc = pos.shape[0]
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(nsrc, self.nbins)
        ev = None if e is None else np.ascontiguousarray(e, dtype=np.float64).reshape(self.nbins)
        if out is None:
            out = dict(Gamma=torch.empty(self.shape, device="cuda"),
                       Heat=torch.empty(self.shape, device="cuda"))
            if segs:
                out["segs"] = torch.empty(self.shape, dtype=torch.int32, device="cuda")
        dp = ctypes.POINTER(ctypes.c_double)
        fn = load().art_point_sources_noalloc if noalloc else load().art_point_sources
        _check(fn(self._h, nsrc, pos.ctypes.data_as(dp), Q.ctypes.data_as(dp),
                                        None if ev is None else ev.ctypes.data_as(dp),
                                        _ptr(n_abs.contiguous()), _ptr(out["Gamma"]),
                                        _ptr(out.get("Heat")), _ptr(out.get("segs")),
                                        _stream_ptr(stream)))
        return out

    def sweep_range(self, nside: int, d_begin: int, d_end: int, I_bc: float = 0.0, A1=None,
                    A2=None, stream=None):
        import torch
        shp = (self.nbins,) + self.shape
        A1 = torch.empty(shp, device="cuda") if A1 is None else A1
        A2 = torch.empty(shp, device="cuda") if A2 is None else A2
        _check(load().art_sweep_range(self._h, nside, d_begin, d_end, float(I_bc), _ptr(A1),
                                      _ptr(A2), _stream_ptr(stream)))
        return A1, A2


def chem_step(n_H, rho, Gamma, Heat, x_HI, u, dt, tables, logT_min, dlogT, T_per_u=1.0, eps=1e-3,
              eps_e=0.2, eps_HI=0.002, max_iter=100, max_sub=100000, dt_chem=None, nsub=None,
              stream=None):
    """art_chem_step on device tensors (n_H, rho, x_HI, u float64; Gamma,
    Heat float32; x_HI and u updated in place).  tables: dict of float64
    device tensors alpha, k_ci, cool_I, cool_II on the log10 T grid."""
    nT = int(tables["alpha"].numel())
    prm = ChemParams(nT, float(logT_min), float(dlogT), *[_ptr(tables[k]) for k in
                     ("alpha", "k_ci", "cool_I", "cool_II")], float(T_per_u), float(eps),
                     float(eps_e), float(eps_HI), int(max_iter), int(max_sub))
    _check(load().art_chem_step(int(n_H.numel()), _ptr(n_H), _ptr(rho), _ptr(Gamma), _ptr(Heat),
                                _ptr(x_HI), _ptr(u), float(dt), ctypes.byref(prm), _ptr(dt_chem),
                                _ptr(nsub), _stream_ptr(stream)))


def release_cost(nwg=40000, words=1024):
    """art_diag_release_cost: ns per workgroup for stores only, a device
    fence, an agent-scope release store, a relaxed store, an acquire load."""
    ns = (ctypes.c_float * 5)()
    _check(load().art_diag_release_cost(int(nwg), int(words), ns))
    return dict(zip(("stores", "fence", "release_store", "relaxed_store", "acquire_load"),
                    [float(v) for v in ns]))


def tune_cache(op: str, path=None):
    """The library's autotune cache: op "clear", "save" or "load" (a text file)."""
    code = {"clear": 0, "save": 1, "load": 2}[op]
    _check(load().art_tune_cache(code, None if path is None else str(path).encode()))


def schedule(shape_xyz, depth=6, subsets=1, waves=1, interleave=3):
    """The block-wavefront schedule of a sweep (art_schedule, host only):
    (items int32 [n, 3] of (wavefront, block, bucket), number of wavefronts)."""
    import numpy as np
    nx, ny, nz = shape_xyz
    t = Tuning(depth, subsets, waves, interleave)
    n = ctypes.c_longlong()
    nw = ctypes.c_int()
    _check(load().art_schedule(nx, ny, nz, ctypes.byref(t), None, 0, ctypes.byref(n), ctypes.byref(nw)))
    items = np.zeros((n.value, 3), dtype=np.int32)
    _check(load().art_schedule(nx, ny, nz, ctypes.byref(t), ctypes.c_void_p(items.ctypes.data),
                               n.value, ctypes.byref(n), ctypes.byref(nw)))
    return items, nw.value


class Batch:
    """Several meshes swept by one graph-captured launch sequence (art_batch_*).

    meshes: list of Mesh (fields set); nsides: list of int; gamma_ws: list of
    per-mesh weight sequences or None.  Output tensors are allocated here and
    kept alive as long as the batch (the graph writes into them)."""

    def __init__(self, meshes, nsides, gamma_ws=None, I_bc: float = 0.0, waves: int = 1,
                 stream=None):
        L = load()
        n = len(meshes)
        self.meshes = list(meshes)
        self.outs = [m.alloc_outputs(ns) for m, ns in zip(meshes, nsides)]
        outs = (Outputs * n)(*[Outputs.of(o) for o in self.outs])
        hs = (ctypes.c_void_p * n)(*[m._h for m in meshes])
        ns_arr = (ctypes.c_int * n)(*[int(v) for v in nsides])
        self._gw_keep = []
        gw_arr = (ctypes.c_void_p * n)()
        for idx in range(n):
            g = None if gamma_ws is None else gamma_ws[idx]
            if g is not None:
                arr = (ctypes.c_float * len(g))(*[float(v) for v in g])
                self._gw_keep.append(arr)
                gw_arr[idx] = ctypes.cast(arr, ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(L.art_batch_create(hs, ns_arr, n, gw_arr, float(I_bc), outs, int(waves),
                                  ctypes.byref(h), _stream_ptr(stream)))
        self._h = h

    def launch(self, stream=None):
        _check(load().art_batch_launch(self._h, _stream_ptr(stream)))
        return self.outs

    def stats(self) -> dict:
        seg = ctypes.c_longlong()
        ms = ctypes.c_float()
        _check(load().art_batch_stats(self._h, ctypes.byref(seg), ctypes.byref(ms)))
        return dict(segment_bins=seg.value, ms=ms.value)

    def close(self):
        if getattr(self, "_h", None):
            load().art_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class nn:
    """Thin wrappers of include/art_nn.h over torch device tensors (argument
    marshalling only; every operation runs in the library's kernels)."""

    @staticmethod
    def _f3(vals):
        return (ctypes.c_float * 3)(*[float(v) for v in vals])

    @staticmethod
    def conv3d_fwd(x, cin, w_k, bias, shape, relu, y=None, y0=None, mask=None, stream=None):
        D, H, W = shape
        _check(load().art_conv3d_fwd(_ptr(x), cin, _ptr(w_k), _ptr(bias), D, H, W, int(relu),
                                     _ptr(mask), _ptr(y), _ptr(y0), _stream_ptr(stream)))

    @staticmethod
    def bwd_weight_workspace(cin, shape):
        """Float32 elements of workspace conv3d_bwd_weight needs."""
        D, H, W = shape
        n = load().art_conv3d_bwd_weight_workspace(cin, D, H, W)
        if n < 0:
            raise ValueError(f"conv3d_bwd_weight: unsupported shape {shape} with cin {cin}")
        return int(n)

    @staticmethod
    def conv3d_bwd_weight(x, cin, g, shape, work, dw, db=None, stream=None):
        D, H, W = shape
        _check(load().art_conv3d_bwd_weight(_ptr(x), cin, _ptr(g), D, H, W, _ptr(work), work.numel(),
                                            _ptr(dw), _ptr(db), _stream_ptr(stream)))

    @staticmethod
    def relu_grad(dy, y, V, g, stream=None):
        _check(load().art_nn_relu_grad(_ptr(dy), _ptr(y), V, _ptr(g), _stream_ptr(stream)))

    @staticmethod
    def prep_weights(w, cin, w_fwd, w_bwd, stream=None):
        _check(load().art_nn_prep_weights(_ptr(w), cin, _ptr(w_fwd), _ptr(w_bwd),
                                          _stream_ptr(stream)))

    @staticmethod
    def mse(pred, target, V, partial, loss, dy, weight=None, stream=None):
        _check(load().art_nn_mse(_ptr(pred), _ptr(target), _ptr(weight), V, _ptr(partial),
                                 _ptr(loss), _ptr(dy), _stream_ptr(stream)))

    @staticmethod
    def sq_weights(J, V, partial, w, lam=0.0, stream=None):
        _check(load().art_nn_sq_weights(_ptr(J), V, float(lam), _ptr(partial), _ptr(w),
                                        _stream_ptr(stream)))

    @staticmethod
    def adamw(w, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0, stream=None):
        _check(load().art_nn_adamw(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), float(lr),
                                   float(beta1), float(beta2), float(eps), float(wd), int(step),
                                   _stream_ptr(stream)))

    @staticmethod
    def features(J, density, x_hi, V, mu, inv_sd, x, stream=None):
        _check(load().art_nn_features(_ptr(J), _ptr(density), _ptr(x_hi), V, nn._f3(mu),
                                      nn._f3(inv_sd), _ptr(x), _stream_ptr(stream)))

    @staticmethod
    def expand(J_coarse, pred, V, J_out, stream=None):
        _check(load().art_nn_expand(_ptr(J_coarse), _ptr(pred), V, _ptr(J_out), _stream_ptr(stream)))

    @staticmethod
    def log_ratio(J_fine, J_coarse, V, target, stream=None):
        _check(load().art_nn_log_ratio(_ptr(J_fine), _ptr(J_coarse), V, _ptr(target),
                                       _stream_ptr(stream)))

    @staticmethod
    def ood_count(x, V, lo, hi, count, stream=None):
        _check(load().art_nn_ood_count(_ptr(x), V, nn._f3(lo), nn._f3(hi), _ptr(count),
                                       _stream_ptr(stream)))


def _farr(vals, nb):
    return None if vals is None else (ctypes.c_float * nb)(*[float(v) for v in vals])


def _rt_chem_args(mesh, n_H, tables, logT_min, dlogT, sigma, src_coef, dalpha, nside, gamma_w, heat_in,
                  heat_src, x_floor, max_iter, T_per_u, eps, eps_e, eps_HI, chem_max_iter, max_sub, sources,
                  work):
    """Parameter blocks of the coupled step (and the host arrays they point
    into, which must stay alive for the call)."""
    import numpy as np
    import torch
    L = load()
    nb = len(sigma)
    if work is None:
        nbytes = L.art_rt_chem_workspace(mesh._h, nb)
        if nbytes < 0:
            raise ValueError("rt_chem_step: bad bin count")
        work = torch.empty(int(nbytes), dtype=torch.uint8, device=n_H.device)
    nT = int(tables["alpha"].numel())
    cp = ChemParams(nT, float(logT_min), float(dlogT), *[_ptr(tables[k]) for k in
                    ("alpha", "k_ci", "cool_I", "cool_II")], float(T_per_u), float(eps), float(eps_e),
                    float(eps_HI), int(chem_max_iter), int(max_sub))
    arrs = [_farr(sigma, nb), _farr(src_coef, nb), _farr(gamma_w, nb), _farr(heat_in, nb), _farr(heat_src, nb)]
    cv = [ctypes.cast(a, ctypes.c_void_p) if a is not None else None for a in arrs]
    nsrc, keep = 0, list(arrs)
    sp = sq = se = None
    if sources is not None:
        pos = np.ascontiguousarray(sources[0], dtype=np.float64).reshape(-1, 3)
        Qa = np.ascontiguousarray(sources[1], dtype=np.float64).reshape(pos.shape[0], nb)
        ea = None if len(sources) < 3 or sources[2] is None else np.ascontiguousarray(sources[2], dtype=np.float64)
        keep += [pos, Qa, ea]
        nsrc = pos.shape[0]
        sp, sq = pos.ctypes.data_as(ctypes.c_void_p), Qa.ctypes.data_as(ctypes.c_void_p)
        se = None if ea is None else ea.ctypes.data_as(ctypes.c_void_p)
    rp = RtChemParams(nb, cv[0], cv[1], _ptr(dalpha), cv[2], cv[3], cv[4], int(nside), float(x_floor),
                      int(max_iter), nsrc, sp, sq, se)
    return rp, cp, work, keep


def rt_chem_step(mesh, n_H, rho, x_HI, u, dt, tables, logT_min, dlogT, sigma, src_coef, dalpha,
                 nside=1, gamma_w=None, heat_in=None, heat_src=None, x_floor=1e-6, max_iter=100,
                 T_per_u=1.0, eps=1e-3, eps_e=0.2, eps_HI=0.002, chem_max_iter=100, max_sub=100000,
                 sources=None, Gamma=None, Heat=None, work=None, stream=None):
    """art_rt_chem_step: one radiative step of `mesh` coupled to the chemistry.
    n_H, rho, x_HI, u: float64 device tensors of the mesh's cells (x_HI, u
    updated in place); tables: float64 device tensors alpha, k_ci, cool_I,
    cool_II; dalpha: float64 device tensor on the same grid; sigma, src_coef
    (and the optional weights): per-bin sequences; sources: None or (pos
    (nsrc, 3), Q (nsrc, nbins), e (nbins,) or None) as for point_sources.
    Returns dict iterations, converged, dt_chem_min."""
    rp, cp, work, keep = _rt_chem_args(mesh, n_H, tables, logT_min, dlogT, sigma, src_coef, dalpha, nside,
                                       gamma_w, heat_in, heat_src, x_floor, max_iter, T_per_u, eps, eps_e,
                                       eps_HI, chem_max_iter, max_sub, sources, work)
    res = RtChemResult()
    _check(load().art_rt_chem_step(mesh._h, ctypes.byref(rp), ctypes.byref(cp), _ptr(n_H), _ptr(rho),
                                   _ptr(x_HI), _ptr(u), float(dt), _ptr(work), int(work.numel()), _ptr(Gamma),
                                   _ptr(Heat), ctypes.byref(res), _stream_ptr(stream)))
    return dict(iterations=res.iterations, converged=bool(res.converged), dt_chem_min=res.dt_chem_min)


def rt_chem_advance(mesh, n_H, rho, x_HI, u, t_end, F, tables, logT_min, dlogT, sigma, src_coef, dalpha,
                    max_steps=100000, nside=1, gamma_w=None, heat_in=None, heat_src=None, x_floor=1e-6,
                    max_iter=100, T_per_u=1.0, eps=1e-3, eps_e=0.2, eps_HI=0.002, chem_max_iter=100,
                    max_sub=100000, sources=None, Gamma=None, Heat=None, work=None, stream=None):
    """art_rt_chem_advance: radiative steps of F chemical timesteps from 0 to
    t_end (arguments as rt_chem_step).  Returns dict steps, iterations,
    unconverged, t, dt_chem_min."""
    rp, cp, work, keep = _rt_chem_args(mesh, n_H, tables, logT_min, dlogT, sigma, src_coef, dalpha, nside,
                                       gamma_w, heat_in, heat_src, x_floor, max_iter, T_per_u, eps, eps_e,
                                       eps_HI, chem_max_iter, max_sub, sources, work)
    run = RtChemRun()
    _check(load().art_rt_chem_advance(mesh._h, ctypes.byref(rp), ctypes.byref(cp), _ptr(n_H), _ptr(rho),
                                      _ptr(x_HI), _ptr(u), float(t_end), float(F), int(max_steps), _ptr(work),
                                      int(work.numel()), _ptr(Gamma), _ptr(Heat), ctypes.byref(run),
                                      _stream_ptr(stream)))
    return dict(steps=run.steps, iterations=run.iterations, unconverged=run.unconverged, t=run.t,
                dt_chem_min=run.dt_chem_min)
