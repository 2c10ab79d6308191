"""Plain FP64 CPU oracle for the HPSCD solver.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the two meet only in the seeded inputs of ``workloads``.

What it computes (paper, Section 2, Algorithm 1 "HPSCD", with the step
derivation of Section 3):

* start from an initial guess a (zero unless given) and the residual
  e = y - X·a (the sign convention of Algorithm 1 and of the nomenclature);
* N cyclic sweeps; in each, for j = 1..n in ascending order:
  da = <X_j, e> / <X_j, X_j>;  e <- e - X_j·da;  a_j <- a_j + da
  (Section 3: the one-column least-squares step, and the residual recursion
  e_{k+1} = e_k - X·da_k);
* both inner products are recomputed at every step, as Algorithm 1 writes them.

Readings where the paper is silent (each is also listed in the design notes):

* a column with <X_j, X_j> = 0 is skipped (da = 0) and counted;
* stopping (Section 2 allows a break once an error is under a threshold, the
  nomenclature calls it max_tol, without defining the error).  After each
  complete sweep s the oracle records hist[s] = ||e||_2 and applies one of
    STOP_NONE        run exactly ``max_sweeps`` sweeps;
    STOP_REL_CHANGE  stop when hist[s-1] - hist[s] < tol * hist[s];
    STOP_REL_RESID   stop when hist[s] < tol * ||y||_2 (also tested before the
                     first sweep, and after every ``check_cols`` column steps
                     when that is positive);
  a zero residual always stops.
* Reduced-precision storage form (``solve_bf16_refresh``): the steps above run
  on X rounded to bfloat16 (round to nearest, ties to even), and every
  ``refresh_cols`` column steps the residual is recomputed exactly as
  e = y - X32·a from the single-precision X.

Parity pins for every function here are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STOP_NONE = 0
STOP_REL_CHANGE = 1
STOP_REL_RESID = 2


@dataclass
class OracleResult:
    a: np.ndarray                 # FP64 coefficients
    e: np.ndarray                 # FP64 running residual
    hist: list                    # ||e||_2 after each complete sweep; hist[0] initial
    sweeps: int                   # complete sweeps performed
    cols: int                     # column steps performed (including skipped columns)
    converged: bool               # a stop test fired
    zero_cols: int                # columns with <X_j, X_j> = 0
    refreshes: int = 0
    extra: dict = field(default_factory=dict)


def _col(Xt, j, m):
    """Column j as FP64 (Xt[j, :m] holds X_j)."""
    return np.asarray(Xt[j, :m], dtype=np.float64)


def residual(Xt, y, m, a):
    """e = y - X·a in FP64 (column by column)."""
    e = np.asarray(y[:m], dtype=np.float64).copy()
    for j in range(len(a)):
        if a[j] != 0.0:
            e -= _col(Xt, j, m) * a[j]
    return e


def final_rel_resid(Xt, y, m, a):
    """||y - X·a||_2 / ||y||_2 evaluated afresh in FP64."""
    ny = np.linalg.norm(np.asarray(y[:m], dtype=np.float64))
    r = np.linalg.norm(residual(Xt, y, m, np.asarray(a, dtype=np.float64)))
    return r / ny if ny > 0 else r


def _sweep_stop(stop, tol, hist, ynorm):
    cur = hist[-1]
    if cur == 0.0:
        return True
    if stop == STOP_REL_CHANGE:
        return (hist[-2] - cur) < tol * cur
    if stop == STOP_REL_RESID:
        return cur < tol * ynorm
    return False


def bf16_round(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    FP32.  bfloat16 keeps the top 16 bits of the binary32 encoding; the low 16
    bits are rounded off with ties going to an even kept part."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_lsb) >> np.uint64(16)) << np.uint64(16)
    r = r.astype(np.uint32)
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    r[nan] = np.uint32(0x7FC00000)
    return r.view(np.float32).reshape(np.shape(x))


def solve(Xt, y, m=None, a0=None, max_sweeps=1, tol=0.0, stop=STOP_NONE,
          check_cols=0, on_step=None, Xt_refresh=None, refresh_cols=0):
    """Algorithm 1 in FP64.

    Xt: (n, >=m) array, Xt[j, :m] = column X_j (any float dtype).
    y: (m,) right-hand side.  a0: optional initial guess.
    on_step(j, e_before, e_after, da, g, d): optional per-step hook.
    Xt_refresh / refresh_cols: when both are given, every ``refresh_cols``
    column steps e is recomputed as y - X_refresh·a (FP64); under
    STOP_REL_RESID a stop that the running residual signals is confirmed on
    a recomputed residual (counted as a refresh) and the sweeps go on from
    that residual when it does not pass.
    Returns an ``OracleResult``.
    """
    n = Xt.shape[0]
    m = Xt.shape[1] if m is None else int(m)
    y64 = np.asarray(y[:m], dtype=np.float64)
    ynorm = float(np.linalg.norm(y64))
    a = np.zeros(n) if a0 is None else np.array(a0, dtype=np.float64)
    e = y64.copy() if a0 is None else residual(Xt if Xt_refresh is None else Xt_refresh, y, m, a)
    hist = [float(np.linalg.norm(e))]
    zero_cols = 0
    for j in range(n):
        x = _col(Xt, j, m)
        if x @ x == 0.0:
            zero_cols += 1
    res = OracleResult(a, e, hist, 0, 0, False, zero_cols)
    confirm = stop == STOP_REL_RESID and bool(refresh_cols) and Xt_refresh is not None

    def passes(nrm):
        return nrm == 0.0 or nrm < tol * ynorm

    def confirmed():
        # reduced-precision form: a stop signalled by the running residual
        # holds only if the residual recomputed from Xt_refresh passes too
        nonlocal e
        e = residual(Xt_refresh, y, m, a)
        res.refreshes += 1
        return passes(float(np.linalg.norm(e)))

    if stop == STOP_REL_RESID and passes(hist[0]) and (not confirm or confirmed()):
        res.converged = True
        return res
    if stop != STOP_NONE and hist[0] == 0.0:
        res.converged = True
        return res
    cols = 0
    for s in range(1, max_sweeps + 1):
        for j in range(n):
            x = _col(Xt, j, m)
            d = x @ x                      # <X_j, X_j>
            if d != 0.0:
                g = x @ e                  # <X_j, e>
                da = g / d
                if on_step is not None:
                    e_before = e.copy()
                e = e - x * da             # e <- e - X_j da
                a[j] = a[j] + da           # a_j <- a_j + da
                if on_step is not None:
                    on_step(j, e_before, e, da, g, d)
            cols += 1
            if refresh_cols and Xt_refresh is not None and cols % refresh_cols == 0:
                e = residual(Xt_refresh, y, m, a)
                res.refreshes += 1
            if (j < n - 1 and check_cols and stop == STOP_REL_RESID
                    and cols % check_cols == 0):
                nrm = float(np.linalg.norm(e))
                if passes(nrm) and (not confirm or confirmed()):
                    res.a, res.e, res.cols, res.sweeps, res.converged = a, e, cols, s - 1, True
                    res.extra["stop_norm"] = nrm
                    return res
        hist.append(float(np.linalg.norm(e)))
        if stop != STOP_NONE and _sweep_stop(stop, tol, hist, ynorm):
            if not confirm or confirmed():
                res.a, res.e, res.cols, res.sweeps, res.converged = a, e, cols, s, True
                return res
            hist[-1] = float(np.linalg.norm(e))
    res.a, res.e, res.cols, res.sweeps = a, e, cols, max_sweeps
    return res


def solve_bf16_refresh(Xt32, y, m=None, a0=None, max_sweeps=1, tol=0.0,
                       stop=STOP_NONE, refresh_cols=0, check_cols=0):
    """The bfloat16-storage form: Algorithm 1 on X rounded to bfloat16, with
    the residual recomputed from the single-precision X every
    ``refresh_cols`` column steps (and e = y - X32·a0 at the start)."""
    Xb = bf16_round(np.asarray(Xt32, dtype=np.float32))
    return solve(Xb, y, m, a0, max_sweeps, tol, stop, check_cols,
                 Xt_refresh=Xt32, refresh_cols=refresh_cols)


def solve_batch(batch, a0pool=None, tols=None, **kw):
    """Solve every system of a packed ``workloads.Batch`` independently;
    ``tols[i] > 0`` replaces ``tol`` for system i."""
    out = []
    for i in range(batch.count):
        s = batch.system(i)
        a_off = int(batch.table[i, 5])
        a0 = None if a0pool is None else a0pool[a_off: a_off + s.n]
        kwi = dict(kw)
        if tols is not None and tols[i] > 0:
            kwi["tol"] = float(tols[i])
        out.append(solve(s.Xt, s.y, s.m, a0, **kwi))
    return out
