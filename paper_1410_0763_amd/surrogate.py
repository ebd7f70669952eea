"""Learned surrogate of the fine sweep (not part of the paper).

A 3-D convolution network (6 layers, 3^3 taps, 32 channels, ReLU between
layers, about 1.1e5 parameters) maps the features of a coarse sweep —
log J at a small HEALPix Nside, log kappa, log S — to log(J_fine / J_coarse),
where J_fine is the mean intensity (eq mean_intensity) of the sweep at a
large Nside.  Every operation runs in the library's kernels (include/art_nn.h:
bf16 matrix-core convolutions with float32 sums, deterministic gradient
reductions, AdamW); this module only allocates device buffers, sequences the
calls, and takes the host-side decisions (training schedule, acceptance
gate, checkpoints).

Acceptance gate: the estimated error of a prediction is the relative L2
error measured on held-out fields after training, plus the fraction of
voxels whose features fall outside the range seen in training; a result is
used only if the estimate is within the caller's bound, otherwise the fine
sweep is run instead (and reported).
"""
from __future__ import annotations

import hashlib
import json
import struct

import numpy as np

from . import art
from .art import nn

CIN = (16, 32, 32, 32, 32, 32)      # input channels of each layer (3 real in layer 0)
REAL_IN = (3, 32, 32, 32, 32, 32)
REAL_OUT = (32, 32, 32, 32, 32, 1)
RELU = (1, 1, 1, 1, 1, 0)
MAGIC = b"ARTSURR1"


class Surrogate:
    """Weights, AdamW state and the device work buffers for one mesh shape."""

    def __init__(self, shape, seed: int = 0, nchunk: int | None = None):
        import torch
        D, H, W = shape
        if W % 32:
            raise ValueError("the surrogate needs the x extent to be a multiple of 32")
        self.shape = (D, H, W)
        self.V = D * H * W
        rows = D * H
        self.nchunk = nchunk or max(c for c in (512, 256, 128, 64, 32, 16, 8, 4, 2, 1) if rows % c == 0)
        self.nchunk_b = max(c for c in (1024, 512, 256, 128, 64, 32, 16, 8, 4, 2, 1) if self.V % c == 0)
        dev = "cuda"
        rng = np.random.default_rng(seed)
        self.w, self.b = [], []
        for l in range(6):
            w = np.zeros((27, CIN[l], 32), np.float32)
            std = np.sqrt(2.0 / (27 * REAL_IN[l])) if l < 5 else 1e-3
            w[:, :REAL_IN[l], :REAL_OUT[l]] = rng.normal(0.0, std, (27, REAL_IN[l], REAL_OUT[l]))
            self.w.append(torch.from_numpy(w).to(dev))
            self.b.append(torch.zeros(32, dtype=torch.float32, device=dev))
        self.mw = [torch.zeros_like(t) for t in self.w]
        self.vw = [torch.zeros_like(t) for t in self.w]
        self.mb = [torch.zeros_like(t) for t in self.b]
        self.vb = [torch.zeros_like(t) for t in self.b]
        self.step = 0
        self.stats = None            # feature normalisation and gate data (set_stats)
        V = self.V
        i16 = torch.int16
        self.w_fwd = [torch.zeros((27, 32, CIN[l]), dtype=i16, device=dev) for l in range(6)]
        self.w_bwd = [torch.zeros((27, 32, 32), dtype=i16, device=dev) for _ in range(6)]
        self.acts = [torch.zeros((V, 32), dtype=i16, device=dev) for _ in range(5)]
        self.pred = torch.zeros(V, dtype=torch.float32, device=dev)
        self.dy = [torch.zeros((V, 32), dtype=i16, device=dev) for _ in range(2)]
        self.g = torch.zeros((V, 32), dtype=i16, device=dev)
        self.gcf = torch.zeros((32, V), dtype=i16, device=dev)
        self.xs = torch.zeros((3, 32, V), dtype=i16, device=dev)
        self.partial = torch.zeros(self.nchunk * 27 * 32 * 32, dtype=torch.float32, device=dev)
        self.bpart = torch.zeros(self.nchunk_b * 32, dtype=torch.float32, device=dev)
        self.dw = [torch.zeros_like(t) for t in self.w]
        self.db = [torch.zeros_like(t) for t in self.b]
        self.mpart = torch.zeros(256, dtype=torch.float32, device=dev)
        self.wpart = torch.zeros(257, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self._prepped = False

    # ------------------------------------------------------------------ #
    def n_params(self) -> int:
        return sum(27 * REAL_IN[l] * REAL_OUT[l] + REAL_OUT[l] for l in range(6))

    def prep(self):
        for l in range(6):
            nn.prep_weights(self.w[l], CIN[l], self.w_fwd[l], self.w_bwd[l])
        self._prepped = True

    def forward(self, x):
        """x: int16 (bf16) [V, 16] features -> self.pred (float32 [V])."""
        if not self._prepped:
            self.prep()
        for l in range(6):
            xin = x if l == 0 else self.acts[l - 1]
            nn.conv3d_fwd(xin, CIN[l], self.w_fwd[l], self.b[l], self.shape, RELU[l],
                          y=self.acts[l] if l < 5 else None, y0=self.pred if l == 5 else None)
        return self.pred

    def gradients(self, x, target, weight=None):
        """Loss (device scalar) and the gradients of every layer into self.dw / self.db."""
        self.prep()
        self.forward(x)
        nn.mse(self.pred, target, self.V, self.mpart, self.loss, self.dy[0], weight=weight)
        cur = 0
        for l in range(5, -1, -1):
            nn.relu_grad(self.dy[cur], self.acts[l] if l < 5 else None, self.V, self.g, self.gcf)
            xin = x if l == 0 else self.acts[l - 1]
            nn.shift3(xin, CIN[l], self.shape, self.xs)
            nn.conv3d_bwd_weight(self.xs, CIN[l], self.gcf, self.shape, self.partial, self.nchunk,
                                 self.dw[l])
            nn.bias_grad(self.gcf, self.V, self.bpart, self.nchunk_b, self.db[l])
            if l > 0:
                nn.conv3d_fwd(self.g, 32, self.w_bwd[l], None, self.shape, 0, y=self.dy[1 - cur])
                cur = 1 - cur
        return self.loss

    def train_step(self, x, target, lr=1e-3, wd=0.0, weight=None):
        loss = self.gradients(x, target, weight)
        self.step += 1
        for l in range(6):
            nn.adamw(self.w[l], self.dw[l], self.mw[l], self.vw[l], lr, self.step, wd=wd)
            nn.adamw(self.b[l], self.db[l], self.mb[l], self.vb[l], lr, self.step)
        self._prepped = False
        return loss

    # ------------------------------------------------------------------ #
    def set_stats(self, mu, sd, lo, hi, val_err=None):
        self.stats = dict(mu=[float(v) for v in mu], sd=[float(v) for v in sd],
                          lo=[float(v) for v in lo], hi=[float(v) for v in hi],
                          val_err=None if val_err is None else float(val_err))

    def features(self, J, kappa, S, x):
        st = self.stats
        nn.features(J, kappa, S, self.V, st["mu"], [1.0 / s for s in st["sd"]], x)

    # ------------------------------------------------------------------ #
    def save(self, path):
        """Weights, AdamW state, step and statistics; the header carries a
        SHA-256 checksum of the binary payload."""
        arrays = [t.cpu().numpy().astype(np.float32) for t in
                  self.w + self.b + self.mw + self.vw + self.mb + self.vb]
        payload = b"".join(a.tobytes() for a in arrays)
        head = dict(shape=list(self.shape), step=self.step, stats=self.stats,
                    sizes=[int(a.size) for a in arrays], sha256=hashlib.sha256(payload).hexdigest())
        hb = json.dumps(head).encode()
        with open(path, "wb") as f:
            f.write(MAGIC + struct.pack("<Q", len(hb)) + hb + payload)

    def load(self, path):
        import torch
        with open(path, "rb") as f:
            data = f.read()
        if data[:8] != MAGIC:
            raise ValueError("not a surrogate checkpoint")
        n = struct.unpack("<Q", data[8:16])[0]
        head = json.loads(data[16:16 + n].decode())
        payload = data[16 + n:]
        if hashlib.sha256(payload).hexdigest() != head["sha256"]:
            raise ValueError("surrogate checkpoint: checksum mismatch")
        if tuple(head["shape"]) != self.shape:
            raise ValueError("surrogate checkpoint: mesh shape differs")
        flat = np.frombuffer(payload, dtype=np.float32)
        off = 0
        targets = self.w + self.b + self.mw + self.vw + self.mb + self.vb
        for t, size in zip(targets, head["sizes"]):
            t.copy_(torch.from_numpy(flat[off:off + size].copy()).reshape(t.shape))
            off += size
        self.step = head["step"]
        self.stats = head["stats"]
        self._prepped = False


def make_pair(mesh, kappa_t, S_t, nside_coarse, nside_fine, model, x, target, weight=None,
              lam=1.0):
    """One training pair on the device: features of the coarse sweep in x,
    log(J_fine / J_coarse) in target, and (if given) the loss weights
    (J_coarse^2 / mean(J_coarse^2) + lam) / (1 + lam) in weight (fields
    already set on mesh)."""
    import torch
    V = model.V
    c = mesh.sweep(nside_coarse)
    f = mesh.sweep(nside_fine)
    Jc = c["J"].reshape(-1)
    Jf = f["J"].reshape(-1)
    model.features(Jc, kappa_t.reshape(-1), S_t.reshape(-1), x)
    nn.log_ratio(Jf, Jc, V, target)
    if weight is not None:
        nn.sq_weights(Jc, V, model.wpart, weight, lam)
    torch.cuda.synchronize()
    return Jc, Jf


def sweep_surrogate(mesh, model, kappa_t, S_t, nside_coarse=2, nside_fine=16, err_bound=0.05,
                    x=None):
    """J at nside_fine from a coarse sweep and the network, or from the fine
    sweep when the gate rejects the prediction.  Returns (J [V] float32,
    used_fallback, est_err)."""
    import torch
    V = model.V
    st = model.stats
    if x is None:
        x = torch.zeros((V, 16), dtype=torch.int16, device="cuda")
    Jc = mesh.sweep(nside_coarse)["J"].reshape(-1)
    model.features(Jc, kappa_t.reshape(-1), S_t.reshape(-1), x)
    nn.ood_count(x, V, st["lo"], st["hi"], model.count)
    model.forward(x)
    J = torch.empty(V, dtype=torch.float32, device="cuda")
    nn.expand(Jc, model.pred, V, J)
    ood = int(model.count.item()) / V
    est = (st["val_err"] if st["val_err"] is not None else float("inf")) + ood
    if err_bound <= 0.0 or not est <= err_bound:
        J = mesh.sweep(nside_fine)["J"].reshape(-1).clone()
        return J, True, est
    return J, False, est
