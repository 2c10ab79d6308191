"""Seeded synthetic systems X·a = y for the solver's workloads.

Every generator uses ``numpy.random.default_rng`` (PCG64) and returns host
arrays.  X is laid out column-major: an array ``Xt`` of shape ``(n, ldx)`` in C
order, whose row ``j`` holds column X_j in its first ``m`` entries.  Rows
``m..ldx-1`` of each column are padding; ``pad`` chooses what they hold (NaN is
used by tests to prove that no kernel reads them).

The workloads stand in for the paper's benchmark systems (Section 9 names tall
and wide single-precision systems but does not describe them):

* ``tall_small``   2000 x 50 Gaussian least squares, noise 0.01
* ``tall_large``   1,000,000 x 256 Gaussian with log-uniform column scales
                   in [0.1, 10], noise 1e-3 (the bandwidth benchmark)
* ``wide``         2000 x 200,000 Gaussian, 1 % sparse a_true, y = X·a_true
* ``batch``        thousands of tall systems, m log-uniform in [256, 8192],
                   n log-uniform in [8, 128], noise 0.01
* ``rbf``          Gaussian radial-basis regression systems, m = 4096, n = 64,
                   with 13 family parameters per system

No function here performs any step of the solver.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "System", "Batch", "round_up", "make_system", "tall_small", "tall_large",
    "wide", "square_well_conditioned", "orthogonal_columns", "batch_sizes",
    "batch", "pack", "rbf_params", "rbf_system", "rbf_features",
    "RBF_NPARAM", "column_orders", "correlated_group",
]


def round_up(x: int, k: int) -> int:
    return (int(x) + k - 1) // k * k


@dataclass
class System:
    """One dense system.  ``Xt[j, :m]`` is column j (float32 unless noted)."""
    Xt: np.ndarray
    y: np.ndarray
    m: int
    n: int
    a_true: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def ldx(self) -> int:
        return self.Xt.shape[1]

    def X(self, dtype=np.float64) -> np.ndarray:
        """Dense (m, n) copy of X in ``dtype`` (for small systems only)."""
        return np.ascontiguousarray(self.Xt[:, : self.m].T, dtype=dtype)


def _alloc_cols(n: int, m: int, ldx: int, pad: float, dtype=np.float32):
    Xt = np.empty((n, ldx), dtype=dtype)
    if ldx > m:
        Xt[:, m:] = pad
    return Xt


def make_system(rng: np.random.Generator, m: int, n: int, *, noise: float,
                col_scale: np.ndarray | None = None, ldx: int | None = None,
                pad: float = 0.0, dtype=np.float32) -> System:
    """Gaussian system.  Draw order: a_true, X (column by column), noise."""
    ldx = round_up(m, 8) if ldx is None else int(ldx)
    a_true = rng.standard_normal(n)
    Xt = _alloc_cols(n, m, ldx, pad, dtype)
    for j in range(n):
        col = rng.standard_normal(m, dtype=np.float32)
        if col_scale is not None:
            col *= np.float32(col_scale[j])
        Xt[j, :m] = col
    y64 = np.zeros(m)
    for j in range(n):  # y = X·a_true, accumulated column by column in FP64
        y64 += Xt[j, :m].astype(np.float64) * a_true[j]
    if noise:
        y64 += noise * rng.standard_normal(m)
    return System(Xt, y64.astype(dtype), m, n, a_true)


def tall_small(seed: int = 1, m: int = 2000, n: int = 50, pad: float = 0.0) -> System:
    """Tall least-squares system, X and a_true iid N(0,1), noise 0.01·N(0,1)."""
    rng = np.random.default_rng(seed)
    s = make_system(rng, m, n, noise=0.01, pad=pad)
    s.meta = dict(workload="tall_small", seed=seed)
    return s


def tall_large(seed: int = 2, m: int = 1_000_000, n: int = 256, pad: float = 0.0) -> System:
    """Tall system with column scales log-uniform in [0.1, 10], noise 1e-3."""
    rng = np.random.default_rng(seed)
    scale = np.exp(rng.uniform(math.log(0.1), math.log(10.0), n))
    s = make_system(rng, m, n, noise=1e-3, col_scale=scale, pad=pad)
    s.meta = dict(workload="tall_large", seed=seed, col_scale=scale)
    return s


def wide(seed: int = 3, m: int = 2000, n: int = 200_000, density: float = 0.01,
         pad: float = 0.0) -> System:
    """Wide consistent system: X iid N(0,1), a_true with ``density`` nonzeros,
    y = X·a_true evaluated in FP64 and rounded to FP32."""
    rng = np.random.default_rng(seed)
    ldx = round_up(m, 8)
    Xt = _alloc_cols(n, m, ldx, pad)
    Xt[:, :m] = rng.standard_normal((n, m), dtype=np.float32)
    nnz = max(1, int(round(density * n)))
    idx = np.sort(rng.choice(n, size=nnz, replace=False))
    a_true = np.zeros(n)
    a_true[idx] = rng.standard_normal(nnz)
    y64 = Xt[idx, :m].astype(np.float64).T @ a_true[idx]
    s = System(Xt, y64.astype(np.float32), m, n, a_true)
    s.meta = dict(workload="wide", seed=seed, nnz=nnz)
    return s


def square_well_conditioned(n: int, seed: int, kind: str = "perturbed_identity") -> System:
    """Consistent square systems with small condition number (y = X·a_true).

    ``perturbed_identity``: X = I + 0.3·G/sqrt(n) with G iid N(0,1).
    ``orth_scaled``: X = Q·diag(U[1,2]) with Q orthogonal (from a QR).
    Values are FP64 (``Xt`` is float64)."""
    rng = np.random.default_rng(seed)
    a_true = rng.standard_normal(n)
    if kind == "perturbed_identity":
        X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / math.sqrt(n)
    elif kind == "orth_scaled":
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        X = Q * rng.uniform(1.0, 2.0, n)
    else:
        raise ValueError(kind)
    Xt = np.ascontiguousarray(X.T)
    return System(Xt, X @ a_true, n, n, a_true, dict(workload=kind, seed=seed))


def orthogonal_columns(m: int, n: int, seed: int) -> System:
    """Tall X with mutually orthogonal columns of different lengths (FP64),
    y iid N(0,1)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    X = Q * rng.uniform(0.5, 3.0, n)
    y = rng.standard_normal(m)
    return System(np.ascontiguousarray(X.T), y, m, n, None,
                  dict(workload="orthogonal_columns", seed=seed))


def column_orders(seed: int, sweeps: int, n: int) -> np.ndarray:
    """Random column orders: row s is a uniformly random permutation of
    0..n-1 (the order of sweep s + 1), int32, shape (sweeps, n)."""
    rng = np.random.default_rng(seed)
    return np.argsort(rng.random((sweeps, n)), axis=1, kind="stable").astype(np.int32)


def correlated_group(m: int, n: int, seed: int, k: int = 3, eps: float = 1e-3,
                     at: int = 0, dtype=np.float32) -> System:
    """Gaussian tall system (noise 0.01) whose columns ``at .. at+k-1`` are
    nearly equal: X_{at+i} = X_at + eps·z_i with z_i iid N(0,1)."""
    rng = np.random.default_rng(seed)
    s = make_system(rng, m, n, noise=0.01, dtype=dtype)
    for i in range(1, k):
        z = rng.standard_normal(m).astype(dtype)
        s.Xt[at + i, :m] = s.Xt[at, :m] + dtype(eps) * z
    y64 = np.zeros(m)
    for j in range(n):
        y64 += s.Xt[j, :m].astype(np.float64) * s.a_true[j]
    s.y = (y64 + 0.01 * rng.standard_normal(m)).astype(dtype)
    s.meta = dict(workload="correlated_group", seed=seed, k=k, eps=eps, at=at)
    return s


# --------------------------------------------------------------------------
# Batches of independent tall systems
# --------------------------------------------------------------------------

@dataclass
class Batch:
    """Packed batch.  ``table[i] = (m, n, x_off, ldx, y_off, a_off)`` in
    elements; column j of system i is ``Xpool[x_off + j*ldx : +m]``."""
    Xpool: np.ndarray
    ypool: np.ndarray
    table: np.ndarray          # int64 (count, 6)
    a_size: int
    a_true: list

    @property
    def count(self) -> int:
        return int(self.table.shape[0])

    def system(self, i: int) -> System:
        m, n, xo, ldx, yo, _ = (int(v) for v in self.table[i])
        Xt = self.Xpool[xo: xo + n * ldx].reshape(n, ldx)
        return System(Xt, self.ypool[yo: yo + m], m, n, self.a_true[i])


def batch_sizes(seed: int, count: int, m_lo: int = 256, m_hi: int = 8192,
                n_lo: int = 8, n_hi: int = 128):
    """Sizes (m_i, n_i): floor of log-uniform draws, forced to n < m."""
    rng = np.random.default_rng(seed)
    ms = np.floor(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))).astype(np.int64)
    ns = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    ns = np.minimum(ns, ms - 1)
    return ms, ns


def batch(seed: int = 4, count: int = 4096, m_lo: int = 256, m_hi: int = 8192,
          n_lo: int = 8, n_hi: int = 128, noise: float = 0.01,
          subset=None, pad: float = 0.0) -> Batch:
    """Batch of independent tall Gaussian systems.  System i draws from its own
    child seed, so any subset is reproducible without drawing the rest."""
    ms, ns = batch_sizes(seed, count, m_lo, m_hi, n_lo, n_hi)
    children = np.random.SeedSequence(seed).spawn(count)
    ids = range(count) if subset is None else list(subset)
    systems = []
    for i in ids:
        rng = np.random.default_rng(children[i])
        systems.append(make_system(rng, int(ms[i]), int(ns[i]), noise=noise, pad=pad))
    return pack(systems)


def pack(systems, align: int = 64) -> Batch:
    """Pack systems into pools; every column starts on a 16-byte boundary and
    every system's X on an ``align``-element boundary."""
    rows, xo, yo, ao = [], 0, 0, 0
    for s in systems:
        xo = round_up(xo, align)
        rows.append((s.m, s.n, xo, s.ldx, yo, ao))
        xo += s.n * s.ldx
        yo += s.m
        ao += s.n
    Xpool = np.zeros(max(xo, 1), dtype=np.float32)
    ypool = np.zeros(max(yo, 1), dtype=np.float32)
    for s, (m, n, x0, ldx, y0, _) in zip(systems, rows):
        Xpool[x0: x0 + n * ldx] = s.Xt.reshape(-1)
        ypool[y0: y0 + m] = s.y
    table = np.array(rows, dtype=np.int64).reshape(-1, 6)
    return Batch(Xpool, ypool, table, ao, [s.a_true for s in systems])


# --------------------------------------------------------------------------
# Parametric radial-basis family (learned warm start workload)
# --------------------------------------------------------------------------

RBF_NPARAM = 13  # sigma, then (A_k, f_k, phi_k) for k = 1..4


def rbf_params(seed: int, count: int, m: int = 4096):
    """Draw ``count`` systems of the RBF family.

    Returns ``(P, T)``: ``P`` (count, 13) FP64 with columns
    ``[sigma, A1..A4, f1..f4, phi1..phi4]``, the four sinusoids sorted by
    frequency (the family is invariant to their order); ``T`` (count, m) FP64
    sample points t_i ~ U[0, 1]."""
    children = np.random.SeedSequence(seed).spawn(count)
    P = np.empty((count, RBF_NPARAM))
    T = np.empty((count, m))
    for i in range(count):
        rng = np.random.default_rng(children[i])
        sigma = rng.uniform(0.02, 0.1)
        A = rng.uniform(0.5, 1.5, 4)
        f = rng.uniform(1.0, 8.0, 4)
        phi = rng.uniform(0.0, 2.0 * math.pi, 4)
        order = np.argsort(f, kind="stable")
        P[i] = np.concatenate([[sigma], A[order], f[order], phi[order]])
        T[i] = rng.uniform(0.0, 1.0, m)
    return P, T


def rbf_system(p: np.ndarray, t: np.ndarray, n: int = 64, ldx: int | None = None,
               dtype=np.float32) -> System:
    """X_ij = exp(-(t_i - c_j)^2 / (2 sigma^2)) with centres c_j = j/(n-1);
    y_i = sum_k A_k sin(2 pi f_k t_i + phi_k).  Evaluated in FP64, stored in
    ``dtype``."""
    m = t.shape[0]
    ldx = round_up(m, 8) if ldx is None else ldx
    sigma, A, f, phi = p[0], p[1:5], p[5:9], p[9:13]
    c = np.arange(n) / (n - 1)
    Xt = np.zeros((n, ldx), dtype=dtype)
    Xt[:, :m] = np.exp(-((t[None, :] - c[:, None]) ** 2) / (2.0 * sigma * sigma))
    y = (A[:, None] * np.sin(2.0 * math.pi * f[:, None] * t[None, :] + phi[:, None])).sum(0)
    return System(Xt, y.astype(dtype), m, n, None, dict(workload="rbf"))


# Network inputs.  Each sinusoid A sin(2 pi f t + phi) is re-coded by its
# phasor (A cos phi, A sin phi): y is linear in the phasors, and the code has
# no jump where phi wraps from 2 pi to 0.  sigma and the sorted f_k are scaled
# from their sampling ranges (uniform on [lo, hi]: mean (lo+hi)/2, std
# (hi-lo)/sqrt(12)); A cos phi and A sin phi have mean 0 and std
# sqrt(E[A^2]/2) = sqrt(13/24) for A ~ U[0.5, 1.5].
_RBF_LO = np.array([0.02] + [1.0] * 4)
_RBF_HI = np.array([0.1] + [8.0] * 4)
_PHASOR_SD = math.sqrt(13.0 / 24.0)


def rbf_features(P: np.ndarray) -> np.ndarray:
    """Network inputs (count, 13) FP32 from family parameters ``P``:
    [sigma, f1..f4, A1 cos phi1, A1 sin phi1, ..., A4 cos phi4, A4 sin phi4],
    each standardised.  A bijective re-coding of the 13 parameters."""
    P = np.asarray(P, dtype=np.float64)
    sf = P[:, [0, 5, 6, 7, 8]]
    mu = 0.5 * (_RBF_LO + _RBF_HI)
    sd = (_RBF_HI - _RBF_LO) / math.sqrt(12.0)
    A, phi = P[:, 1:5], P[:, 9:13]
    ph = np.empty((len(P), 8))
    ph[:, 0::2] = A * np.cos(phi)
    ph[:, 1::2] = A * np.sin(phi)
    return np.concatenate([(sf - mu) / sd, ph / _PHASOR_SD], axis=1).astype(np.float32)
