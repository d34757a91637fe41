"""Training driver of the learned Newton guess.

Torch holds the buffers (FP32 master parameters, their BF16 copy, Adam
moments, gradients, activation cache) and draws the mini-batch indices; the
forward pass, the loss gradient, the backward pass and the Adam update are
the library's HIP kernels (srmhd_mlp_*), with every matrix product on the
matrix cores in BF16 with FP32 accumulation.
"""
from __future__ import annotations

import math

import torch

from . import binding as B


class Mlp:
    def __init__(self, seed=0, device="cuda"):
        self.device = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        p = torch.zeros(B.MLP_NPARAM, dtype=torch.float32)
        # He-uniform initial weights, zero biases
        for name, (rows, cols) in {"W1": (64, 5), "W2": (64, 64), "W3": (2, 64)}.items():
            o = B.MLP_OFF[name]
            lim = math.sqrt(6.0 / cols)
            p[o:o + rows * cols] = (torch.rand(rows * cols, generator=g) * 2 - 1) * lim
        self.params = p.to(self.device)
        self.w = torch.empty(B.MLP_NPARAM, dtype=torch.bfloat16, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.t = 0
        self.norm = [0.0] * 5 + [1.0] * 5 + [0.0, 0.0, 1.0, 1.0]
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._cache = None
        self._batch = 0
        self.quantize()

    @property
    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def quantize(self):
        B.srmhd_mlp_quantize(self.params.data_ptr(), self.w.data_ptr(), B.MLP_NPARAM, self.stream)

    def _ensure_cache(self, batch):
        if self._cache is None or self._batch != batch:
            nb = B.srmhd_mlp_cache_bytes(batch)
            if nb == 0:
                raise ValueError(f"batch {batch} out of range")
            buf = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            self._cache, self._cache_ptr, self._batch = buf, buf.data_ptr() + off, batch

    # -------------------------------------------------------------- kernels
    def forward(self, x):
        """x (batch, 5) standardised features -> y (batch, 2)."""
        x = x.contiguous().float()
        n = x.shape[0]
        self._ensure_cache(n)
        y = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        B.srmhd_mlp_forward(self.params.data_ptr(), self.w.data_ptr(), x.data_ptr(), y.data_ptr(),
                            self._cache_ptr, n, self.stream)
        return y

    def loss_and_grad(self, x, t):
        """Loss (device scalar) and self.grad for one batch."""
        y = self.forward(x)
        t = t.contiguous().float()
        B.srmhd_mlp_loss_grad(y.data_ptr(), t.data_ptr(), self._cache_ptr, self._loss.data_ptr(),
                              x.shape[0], self.stream)
        B.srmhd_mlp_backward(self.w.data_ptr(), self._cache_ptr, self.grad.data_ptr(),
                             x.shape[0], self.stream)
        return self._loss

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        B.srmhd_mlp_adam(self.params.data_ptr(), self.w.data_ptr(), self.m.data_ptr(),
                         self.v.data_ptr(), self.grad.data_ptr(), B.MLP_NPARAM, lr, beta1, beta2,
                         eps, self.t, self.stream)

    # ------------------------------------------------------------- training
    def set_normalisation(self, feats, targets):
        fm, fs = feats.mean(0), feats.std(0).clamp_min(1e-6)
        tm, ts = targets.mean(0), targets.std(0).clamp_min(1e-6)
        self.norm = [*fm.tolist(), *fs.tolist(), *tm.tolist(), *ts.tolist()]

    def standardise(self, feats, targets=None):
        n = torch.tensor(self.norm, dtype=torch.float32, device=feats.device)
        x = (feats - n[0:5]) / n[5:10]
        if targets is None:
            return x
        return x, (targets - n[10:12]) / n[12:14]

    def fit(self, feats, targets, steps=2000, batch=4096, lr=1e-3, seed=1, log_every=0):
        """Adam on the MSE of the standardised targets; returns the loss history."""
        self.set_normalisation(feats, targets)
        x_all, t_all = self.standardise(feats, targets)
        g = torch.Generator(device=self.device).manual_seed(seed)
        batch = min(batch, x_all.shape[0])
        hist = []
        for s in range(steps):
            idx = torch.randint(0, x_all.shape[0], (batch,), generator=g, device=self.device)
            loss = self.loss_and_grad(x_all[idx], t_all[idx])
            self.adam_step(lr)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist

    def predict(self, feats):
        """De-standardised (log(p/D), log Gamma) for raw features."""
        n = torch.tensor(self.norm, dtype=torch.float32, device=self.device)
        y = self.forward(self.standardise(feats))
        return y * n[12:14] + n[10:12]


def harvest_training_set(device="cuda", turb_n=64, sigmas=(1.0, 3.0, 10.0), gamma_max=5.0,
                         snapshots=4, steps_between=3, frac=0.05, seed=10):
    """(features, targets) harvested by the solver itself: the CPA waves on
    the axis and the diagonal at 32^3, and the turbulence set-up at turb_n^3
    for each magnetisation in `sigmas`, at `snapshots` times a few steps
    apart."""
    from . import inputs
    from .solver import Solver
    feats, targs = [], []
    for diag in (False, True):
        prim5, bf, _ = inputs.cpa(32, diagonal=diag)
        S = Solver(32, device=device)
        S.init(prim5, bf)
        S.step(2)
        f, t = S.harvest(4096, 0.1, seed=1)
        feats.append(f)
        targs.append(t)
        S.close()
    cap = int(turb_n ** 3 * frac * 1.3) + 64
    for sig in sigmas:
        prim5, bf = inputs.turbulence(turb_n, sigma0=sig, gamma_max=gamma_max, device=device)
        S = Solver(turb_n, pfloor=1e-10, device=device)
        S.init(prim5, bf)
        for k in range(snapshots):
            f, t = S.harvest(cap, frac, seed=seed + k)
            feats.append(f)
            targs.append(t)
            S.step(steps_between)
        S.close()
    return torch.cat(feats), torch.cat(targs)


def train_default(device="cuda", steps=1500, seed=0):
    """The network used by the learned form: trained on harvest_training_set()."""
    feats, targs = harvest_training_set(device)
    mlp = Mlp(seed=seed, device=device)
    hist = mlp.fit(feats, targs, steps=steps, batch=4096, lr=2e-3, seed=1, log_every=250)
    return mlp, hist, feats.shape[0]
