"""Bulk construction of the radial-basis family on a torch device.

The learned warm start trains on tens of thousands of these systems (1 MiB
of X each at m = 4096, n = 64), too many to build on the host and copy.  This
module evaluates the same formulas as ``gen.rbf_system`` (FP64 arithmetic,
stored FP32) with torch tensor operations on any device, and packs the
systems into the pool layout of the batched solver.  It performs no step of
the solver.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = ["rbf_pool"]


def rbf_pool(P, T, n: int = 64, device="cpu", chunk: int = 512):
    """Systems i = 0..count-1 from parameters ``P`` (count, 13) and sample
    points ``T`` (count, m), as returned by ``gen.rbf_params``.

    Returns ``(Xpool, ypool, table)``: FP32 tensors on ``device`` with system
    i's column-major X (ldx = m) at ``x_off = i*n*m`` and y at ``y_off = i*m``,
    and the int64 table rows ``(m, n, x_off, ldx, y_off, a_off = i*n)``."""
    P = np.asarray(P, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    count, m = T.shape
    if m % 4:
        raise ValueError("m must be a multiple of 4 (16-byte aligned columns)")
    Xpool = torch.empty(count * n * m, dtype=torch.float32, device=device)
    ypool = torch.empty(count * m, dtype=torch.float32, device=device)
    c = torch.arange(n, dtype=torch.float64, device=device) / (n - 1)
    for s0 in range(0, count, chunk):
        s1 = min(count, s0 + chunk)
        p = torch.as_tensor(P[s0:s1], device=device)
        t = torch.as_tensor(T[s0:s1], device=device)
        sigma = p[:, 0]
        X = torch.exp(-((t[:, None, :] - c[None, :, None]) ** 2) / (2.0 * sigma[:, None, None] * sigma[:, None, None]))
        Xpool[s0 * n * m: s1 * n * m] = X.reshape(-1).to(torch.float32)
        A, f, phi = p[:, 1:5], p[:, 5:9], p[:, 9:13]
        terms = A[:, :, None] * torch.sin(2.0 * math.pi * f[:, :, None] * t[:, None, :] + phi[:, :, None])
        y = ((terms[:, 0] + terms[:, 1]) + terms[:, 2]) + terms[:, 3]
        ypool[s0 * m: s1 * m] = y.reshape(-1).to(torch.float32)
    i = np.arange(count, dtype=np.int64)
    table = np.stack([np.full(count, m), np.full(count, n), i * n * m, np.full(count, m), i * m, i * n], axis=1)
    return Xpool, ypool, table.astype(np.int64)
