"""Learned warm start for parametric families of systems.

Algorithm 1 (Section 2) may start from any initial guess a0; its sweeps then
work on the residual y - X·a0 (Section 3).  For a family of systems indexed by
a few parameters, a perceptron trained on the solver's own solutions predicts
a0 from the parameters, and the solve from a0 needs fewer sweeps to reach the
residual that a solve from zero reaches after K sweeps.

Training labels are the solver's K-sweep iterates from zero (batched solve),
the network is trained by the library's forward/backward/Adam kernels, and
inference is one forward launch followed by a batched solve from a0.  This
module only moves tensors between those calls; it never does the arithmetic
of the solver or of the network itself.  The solve from zero remains the
fallback: a0 only changes where the iteration starts, and the final FP64
check of every solve judges the result.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import hpscd


def _torch():
    import torch
    return torch


@dataclass
class Labels:
    a: object            # (count, n) FP32 device tensor: the K-sweep iterates from zero
    tau: np.ndarray      # ||e_K|| / ||y|| reached by those iterates (running residual)
    sweeps: int


def label(Xpool, ypool, table, K: int = 100) -> Labels:
    """Run K sweeps from zero on every system of the pool (one batched launch)
    and return the iterates and the relative residual each one reached."""
    table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
    n = int(table[0, 1])
    if not np.all(table[:, 1] == n) or not np.all(table[:, 5] == np.arange(len(table)) * n):
        raise ValueError("labels need systems of equal n with a_off = i*n")
    r = hpscd.solve_batched(Xpool, ypool, table, max_sweeps=K, stop=hpscd.STOP_NONE, want_hist=True,
                            flags=hpscd.F_NO_FINAL_CHECK)
    tau = r.hist[:, K] / r.hist[:, 0]
    return Labels(r.a.view(len(table), n), tau, K)


class WarmStart:
    """Perceptron n_in -> h1 -> h2 -> n_out whose output is an initial guess."""

    def __init__(self, n_in: int, n_out: int, hidden=(256, 256), device: int | None = None, seed: int = 0):
        torch = _torch()
        self.shape = (int(n_in), int(hidden[0]), int(hidden[1]), int(n_out))
        self.net = hpscd.MLP(*self.shape, device=device)
        self.device = torch.device("cuda", self.net.device)
        self.set_params(torch.from_numpy(self.init_params(self.shape, seed)).to(self.device))

    @staticmethod
    def init_params(shape, seed: int) -> np.ndarray:
        """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, in the
        library's flat layout."""
        rng = np.random.default_rng(seed)
        n_in, h1, h2, n_out = shape
        parts = []
        for fan_in, rows in ((n_in, h1), (h1, h2), (h2, n_out)):
            b = 1.0 / math.sqrt(fan_in)
            parts.append(rng.uniform(-b, b, rows * fan_in))
            parts.append(rng.uniform(-b, b, rows))
        return np.concatenate(parts).astype(np.float32)

    def set_params(self, flat):
        self.net.set_params(flat.contiguous())

    def params(self):
        return self.net.get_params()

    def fit(self, feats, targets, *, epochs: int = 100, batch: int = 256, lr: float = 1e-3,
            lr_final: float | None = None, seed: int = 0, log_every: int = 0):
        """Train on (feats, targets) with Adam on the mean squared error, the
        step size decaying from lr to lr_final (default lr/100) on a cosine
        over the epochs.  The targets are standardised per output for training;
        the scaling is folded into the last layer afterwards, so predict()
        returns targets directly.  Returns the first-batch loss of each epoch
        (standardised units)."""
        torch = _torch()
        N = feats.shape[0]
        mu = targets.mean(0)
        sd = targets.std(0).clamp_min(1e-12)
        Ts = ((targets - mu) / sd).contiguous()
        gen = torch.Generator().manual_seed(seed)
        hist = []
        lr_final = lr / 100.0 if lr_final is None else lr_final
        for ep in range(epochs):
            lr_ep = lr_final + (lr - lr_final) * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs)))
            perm = torch.randperm(N, generator=gen).to(self.device)
            xs, ts = feats[perm].contiguous(), Ts[perm].contiguous()
            losses = []
            for b0 in range(0, N, batch):
                b1 = min(N, b0 + batch)
                want = b0 == 0
                L = self.net.train_step(xs[b0:b1], ts[b0:b1], lr_ep, want_loss=want)
                if want:
                    losses.append(L)
            hist.append(float(np.mean(losses)))
            if log_every and (ep + 1) % log_every == 0:
                print(f"epoch {ep + 1}: loss {hist[-1]:.4g}", flush=True)
        self._fold_output_scaling(mu, sd)
        return hist

    def _fold_output_scaling(self, mu, sd):
        """o = sd * (W3 h + b3) + mu  ==  (sd W3) h + (sd b3 + mu)."""
        n_in, h1, h2, n_out = self.shape
        p = self.params()
        w3 = p.numel() - n_out - n_out * h2
        p[w3: w3 + n_out * h2] = (p[w3: w3 + n_out * h2].view(n_out, h2) * sd[:, None]).reshape(-1)
        p[-n_out:] = p[-n_out:] * sd + mu
        self.set_params(p)

    def predict(self, feats, out=None):
        """Initial guesses (count, n_out) for the systems with these features
        (written into ``out`` when given, e.g. the a0 pool of a BatchPlan)."""
        return self.net.forward(feats.contiguous(), out=out)

    def save(self, path: str):
        np.savez(path, shape=np.asarray(self.shape, dtype=np.int64), params=self.params().cpu().numpy())

    @classmethod
    def load(cls, path: str, device: int | None = None) -> "WarmStart":
        torch = _torch()
        with np.load(path, allow_pickle=False) as z:
            shape = tuple(int(v) for v in z["shape"])
            params = z["params"].astype(np.float32)
        ws = cls(shape[0], shape[3], hidden=shape[1:3], device=device)
        ws.set_params(torch.from_numpy(params).to(ws.device))
        return ws


def solve_from(Xpool, ypool, table, a0=None, *, tols, max_sweeps: int):
    """Batched solve of every system until ||e|| < tols[i]·||y|| (at most
    max_sweeps sweeps), from a0 (count, n) or from zero."""
    a0pool = None if a0 is None else a0.reshape(-1).contiguous()
    return hpscd.solve_batched(Xpool, ypool, table, a0pool, max_sweeps=max_sweeps, stop=hpscd.STOP_REL_RESID,
                               tols=tols)
