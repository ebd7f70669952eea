"""Python binding of the learned surrogate (include/art_surrogate.h):
argument marshalling only.

The surrogate is a 3-D convolution network (6 layers, 3^3 taps, 32 channels,
about 1.1e5 parameters) that maps a coarse sweep's log J plus the log density
and the neutral fraction to log(J_in,fine / J_in,coarse), J_in being the
incoming part of J = J_in + S.  Its parameters, optimiser state, work
buffers, training step, inference, acceptance gate with fallback to the fine
sweep, and checkpoints all live in the HIP library; torch tensors serve as
device buffers and torch streams as HIP streams.  The surrogate is not part of
the paper; it stands in for the fine sweep of Sect. 2.2-2.3.
"""
from __future__ import annotations

import ctypes
import math

from . import art
from .art import Outputs, _check, _ptr, _stream_ptr, load

W, B, DW, DB = 0, 1, 2, 3          # parameter arrays of Surrogate.param
CIN = (16, 32, 32, 32, 32, 32)     # stored input channels of each layer


def _f3(vals):
    return (ctypes.c_float * 3)(*[float(v) for v in vals])


class Surrogate:
    """Library-owned network for meshes of shape (D, H, W), W a multiple of 32."""

    def __init__(self, shape, seed: int = 0):
        import torch
        D, H, Wx = shape
        h = ctypes.c_void_p()
        _check(load().art_surrogate_create(Wx, H, D, int(seed), ctypes.byref(h)))
        self._h = h
        self.shape = (D, H, Wx)
        self.V = D * H * Wx
        self.pred = torch.zeros(self.V, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def close(self):
        if getattr(self, "_h", None):
            load().art_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n_params(self) -> int:
        return _check_count(load().art_surrogate_n_params(self._h))

    # -- statistics and gate data -----------------------------------------
    def set_stats(self, mu, sd, lo, hi, val_err=None):
        ve = -1.0 if val_err is None else float(val_err)
        _check(load().art_surrogate_set_stats(self._h, _f3(mu), _f3(sd), _f3(lo), _f3(hi), ve))

    @property
    def stats(self) -> dict:
        a = [(ctypes.c_float * 3)() for _ in range(4)]
        ve = ctypes.c_float()
        _check(load().art_surrogate_get_stats(self._h, *a, ctypes.byref(ve)))
        mu, sd, lo, hi = ([float(v) for v in x] for x in a)
        return dict(mu=mu, sd=sd, lo=lo, hi=hi,
                    val_err=None if math.isnan(ve.value) else float(ve.value))

    def set_val_err(self, val_err):
        st = self.stats
        self.set_stats(st["mu"], st["sd"], st["lo"], st["hi"], val_err)

    def fit_stats(self, J_coarse, density, x_hi, margin: float = 1.0, stream=None):
        """Statistics from lists of device float32 [V] tensors (synchronises)."""
        n = len(J_coarse)
        arrs = [(ctypes.c_void_p * n)(*[t.data_ptr() for t in ts]) for ts in (J_coarse, density, x_hi)]
        _check(load().art_surrogate_fit_stats(self._h, n, *arrs, float(margin),
                                              _stream_ptr(stream)))

    def features(self, J, density, x_hi, x, stream=None):
        _check(load().art_surrogate_features(self._h, _ptr(J), _ptr(density), _ptr(x_hi), _ptr(x),
                                             _stream_ptr(stream)))

    # -- training and inference -------------------------------------------
    def gradients(self, x, target, weight=None, stream=None):
        _check(load().art_surrogate_gradients(self._h, _ptr(x), _ptr(target), _ptr(weight),
                                              _ptr(self.loss), _stream_ptr(stream)))
        return self.loss

    def train_step(self, x, target, lr=1e-3, wd=0.0, weight=None, stream=None):
        _check(load().art_surrogate_train_step(self._h, _ptr(x), _ptr(target), _ptr(weight),
                                               float(lr), float(wd), _ptr(self.loss),
                                               _stream_ptr(stream)))
        return self.loss

    def forward(self, x, stream=None):
        _check(load().art_surrogate_infer(self._h, _ptr(x), _ptr(self.pred), _stream_ptr(stream)))
        return self.pred

    def param(self, layer: int, what: int, stream=None):
        import torch
        n = 27 * CIN[layer] * 32 if what in (W, DW) else 32
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(load().art_surrogate_param(self._h, layer, what, _ptr(t), 0, _stream_ptr(stream)))
        return t.reshape(27, CIN[layer], 32) if what in (W, DW) else t

    def set_param(self, layer: int, what: int, t, stream=None):
        t = t.contiguous()
        _check(load().art_surrogate_param(self._h, layer, what, _ptr(t), 1, _stream_ptr(stream)))

    # -- checkpoints --------------------------------------------------------
    def save(self, path, stream=None):
        _check(load().art_surrogate_save(self._h, str(path).encode(), _stream_ptr(stream)))

    def load(self, path, stream=None):
        _check(load().art_surrogate_load(self._h, str(path).encode(), _stream_ptr(stream)))


def _check_count(rc):
    if rc < 0:
        _check(rc)
    return rc


def make_pair(mesh, model, nside_coarse, nside_fine, target, weight=None, J_coarse=None,
              J_fine=None, lam=1.0, stream=None):
    """Training pair of the field loaded in mesh: target = log(J_in,fine /
    J_in,coarse) and the loss weights (art_surrogate_make_pair).  Returns
    (J_coarse, J_fine) device tensors [V]."""
    import torch
    V = model.V
    Jc = torch.empty(V, dtype=torch.float32, device="cuda") if J_coarse is None else J_coarse
    Jf = torch.empty(V, dtype=torch.float32, device="cuda") if J_fine is None else J_fine
    _check(load().art_surrogate_make_pair(model._h, mesh._h, nside_coarse, nside_fine, float(lam),
                                          _ptr(target), _ptr(weight), _ptr(Jc), _ptr(Jf),
                                          _stream_ptr(stream)))
    return Jc, Jf


def sweep_surrogate(mesh, model, density, x_hi, nside_coarse=2, nside_fine=16, err_bound=0.05,
                    gamma_w=None, out=None, stream=None):
    """art_sweep_surrogate for the field in mesh made from density and x_hi
    (device float32 tensors of the mesh's cells): returns (outputs dict,
    used_fallback, est_err)."""
    if out is None:
        out = mesh.alloc_outputs(nside_fine)
    o = Outputs.of({k: v for k, v in out.items() if k != "exit_sum"})
    gw = None
    if gamma_w is not None:
        arr = (ctypes.c_float * 1)(float(gamma_w[0]))
        gw = ctypes.cast(arr, ctypes.c_void_p)
    fb = ctypes.c_int()
    est = ctypes.c_float()
    _check(load().art_sweep_surrogate(mesh._h, model._h, _ptr(density.contiguous()),
                                      _ptr(x_hi.contiguous()), nside_coarse, nside_fine, gw,
                                      float(err_bound), ctypes.byref(o), ctypes.byref(fb),
                                      ctypes.byref(est), _stream_ptr(stream)))
    return out, bool(fb.value), float(est.value)


def sha256(data: bytes) -> bytes:
    """Digest of the checkpoint format, computed by the library."""
    buf = ctypes.create_string_buffer(bytes(data), max(len(data), 1))
    dig = (ctypes.c_ubyte * 32)()
    _check(load().art_sha256(buf, len(data), dig))
    return bytes(dig)


__all__ = ["Surrogate", "make_pair", "sweep_surrogate", "sha256", "W", "B", "DW", "DB", "art"]
