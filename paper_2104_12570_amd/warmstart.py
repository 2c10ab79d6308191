"""Learned warm start for parametric families of systems.

Algorithm 1 (Section 2) may start from any initial guess a0; its sweeps then
work on the residual y - X·a0 (Section 3).  For a family of systems indexed by
a few parameters, a perceptron trained on the solver's own solutions predicts
a0 from the parameters, and the solve from a0 needs fewer sweeps to reach the
residual that a solve from zero reaches after K sweeps.

Training labels are the solver's K-sweep iterates from zero (batched solve),
the network is trained by the library's forward/backward/Adam kernels, and
inference is one forward launch followed by a batched solve from a0.  This
module only sequences those calls and indexes or moves tensors between them;
it never does the arithmetic of the solver or of the network itself.  The
solve from zero remains the fallback: every system that the initial guess
did not bring to its tolerance is solved again from zero, and the final FP64
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
        # parameters drawn by the library (uniform in +-1/sqrt(fan_in), seeded)
        self.net = hpscd.MLP(*self.shape, device=device, seed=seed)
        self.device = torch.device("cuda", self.net.device)

    def set_params(self, flat):
        self.net.set_params(flat.contiguous())

    def params(self):
        return self.net.get_params()

    def fit(self, feats, targets, *, epochs: int = 100, batch: int = 256, lr: float = 1e-3,
            lr_final: float | None = None, seed: int = 0, log_every: int = 0):
        """Train on (feats, targets) with Adam on the mean squared error, the
        step size decaying from lr to lr_final (default lr/100) on a cosine
        over the epochs.  The library standardises the targets per output
        (hpscd_mlp_fit_output_scaling) and returns predictions in target units.
        Returns the first-batch loss of each epoch (standardised units)."""
        torch = _torch()
        N = feats.shape[0]
        targets = targets.contiguous()
        self.net.fit_output_scaling(targets)
        gen = torch.Generator().manual_seed(seed)
        hist = []
        lr_final = lr / 100.0 if lr_final is None else lr_final
        for ep in range(epochs):
            lr_ep = lr_final + (lr - lr_final) * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs)))
            perm = torch.randperm(N, generator=gen).to(self.device)
            xs, ts = feats[perm].contiguous(), targets[perm].contiguous()
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
        return hist

    def predict(self, feats, out=None):
        """Initial guesses (count, n_out) for the systems with these features
        (written into ``out`` when given, e.g. the a0 pool of a BatchPlan)."""
        return self.net.forward(feats.contiguous(), out=out)

    def save(self, path: str):
        np.savez(path, shape=np.asarray(self.shape, dtype=np.int64), params=self.params().cpu().numpy(),
                 scaling=self.net.output_scaling().cpu().numpy())

    @classmethod
    def load(cls, path: str, device: int | None = None) -> "WarmStart":
        torch = _torch()
        with np.load(path, allow_pickle=False) as z:
            shape = tuple(int(v) for v in z["shape"])
            params = z["params"].astype(np.float32)
            scaling = z["scaling"].astype(np.float32)
        ws = cls(shape[0], shape[3], hidden=shape[1:3], device=device)
        ws.set_params(torch.from_numpy(params).to(ws.device))
        ws.net.set_output_scaling(torch.from_numpy(scaling).to(ws.device))
        return ws


@dataclass
class WarmResult:
    a: object                 # (count * n,) FP32 device tensor: every system's result
    sweeps: np.ndarray        # sweeps of the warm solve (plus those of the fallback where it ran)
    converged: np.ndarray     # each system reached its tolerance
    fallback: np.ndarray      # indices of the systems re-solved from zero
    final_rel_resid: np.ndarray


def solve_from(Xpool, ypool, table, a0=None, *, tols, max_sweeps: int, fallback: bool = True) -> WarmResult:
    """Batched solve of every system until ||e|| < tols[i]·||y|| (at most
    max_sweeps sweeps), from a0 (count, n) or from zero.  With ``fallback``,
    every system that a0 did not bring to its tolerance is solved again from
    zero (one more batched launch over those systems): the solve from zero is
    the result of record wherever the initial guess did not pay off."""
    torch = _torch()
    table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
    tols = np.asarray(tols, dtype=np.float64).reshape(-1)
    a0pool = None if a0 is None else a0.reshape(-1).contiguous()
    r = hpscd.solve_batched(Xpool, ypool, table, a0pool, max_sweeps=max_sweeps, stop=hpscd.STOP_REL_RESID,
                            tols=tols)
    a = r.a
    sweeps, conv, fr = r.sweeps.copy(), r.converged.copy(), r.final_rel_resid.copy()
    missed = np.flatnonzero(conv == 0) if (fallback and a0 is not None) else np.zeros(0, np.int64)
    if missed.size:
        sub = table[missed]
        r0 = hpscd.solve_batched(Xpool, ypool, sub, None, max_sweeps=max_sweeps, stop=hpscd.STOP_REL_RESID,
                                 tols=tols[missed], a_size=a.numel())
        idx = torch.from_numpy(np.concatenate([np.arange(o, o + k) for o, k in zip(sub[:, 5], sub[:, 1])]))
        idx = idx.to(a.device)
        a[idx] = r0.a[idx]
        sweeps[missed] += r0.sweeps
        conv[missed] = r0.converged
        fr[missed] = r0.final_rel_resid
    return WarmResult(a, sweeps, conv, missed, fr)
