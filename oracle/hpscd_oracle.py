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
    STOP_REL_GRAD    stop when ||X^T e||_2 < tol * ||X^T y||_2 after a sweep
                     (the gradient of ||e||^2 / 2 relative to its value at
                     a = 0; for least-squares systems, whose residual never
                     reaches zero);
  a zero residual (or, under STOP_REL_GRAD, a zero gradient) always stops.
* Column order (Section 2 names a randomly selected index as a variation):
  ``order`` gives the columns visited in each sweep, one permutation per
  sweep; the default is the cyclic ascending order of Algorithm 1.
* Reduced-precision storage form (``solve_bf16_refresh``): the steps above run
  on X rounded to bfloat16 (round to nearest, ties to even), and every
  ``refresh_cols`` column steps the residual is recomputed exactly as
  e = y - X32·a from the single-precision X.
* ``solve_parallel``: the parallel solver of Section 7 (Algorithm 2), blocks
  of ``thr`` columns whose steps all use the residual of the block start.
* ``select_features``: the feature-selection variant of Section 8
  (Algorithm 3), greedy selection of the column that most reduces ||e||.

Parity pins for every function here are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STOP_NONE = 0
STOP_REL_CHANGE = 1
STOP_REL_RESID = 2
STOP_REL_GRAD = 3


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


def gradient(Xt, m, e):
    """X^T e in FP64, one inner product per column (the gradient of
    ||e||^2 / 2 with respect to a, up to its sign)."""
    return np.array([_col(Xt, j, m) @ e for j in range(Xt.shape[0])])


# The three lines of Algorithm 1's inner loop, kept as separate functions so
# that a test can plant a mistake in any one of them.
def _step_size(x, e, d):
    """da = <X_j, e> / <X_j, X_j>."""
    return (x @ e) / d


def _residual_update(e, x, da):
    """e <- e - X_j da."""
    return e - x * da


def _coef_update(a, j, da):
    """a_j <- a_j + da."""
    a[j] = a[j] + da


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
          check_cols=0, on_step=None, Xt_refresh=None, refresh_cols=0, order=None):
    """Algorithm 1 in FP64.

    Xt: (n, >=m) array, Xt[j, :m] = column X_j (any float dtype).
    y: (m,) right-hand side.  a0: optional initial guess.
    on_step(j, e_before, e_after, da, g, d): optional per-step hook.
    Xt_refresh / refresh_cols: when both are given, every ``refresh_cols``
    column steps e is recomputed as y - X_refresh·a (FP64); under
    STOP_REL_RESID a stop that the running residual signals is confirmed on
    a recomputed residual (counted as a refresh) and the sweeps go on from
    that residual when it does not pass.
    order: None (cyclic, j = 1..n) or an integer array (>= max_sweeps, n)
    whose row s-1 lists the columns visited in sweep s.
    Under STOP_REL_GRAD, ``extra["grad_hist"][s]`` = ||X^T e|| after sweep s
    (index 0: before the first sweep) and ``extra["xty_norm"]`` = ||X^T y||.
    Returns an ``OracleResult``.
    """
    n = Xt.shape[0]
    m = Xt.shape[1] if m is None else int(m)
    if order is not None:
        order = np.asarray(order)
        if order.ndim != 2 or order.shape[1] != n or order.shape[0] < max_sweeps:
            raise ValueError("order must have shape (>= max_sweeps, n)")
        for s in range(max_sweeps):
            if not np.array_equal(np.sort(order[s]), np.arange(n)):
                raise ValueError(f"order row {s} is not a permutation of 0..n-1")
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
    if stop == STOP_REL_GRAD:
        xty = float(np.linalg.norm(gradient(Xt, m, y64)))
        res.extra["xty_norm"] = xty
        res.extra["grad_hist"] = [float(np.linalg.norm(gradient(Xt, m, e)))]

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
        for k in range(n):
            j = k if order is None else int(order[s - 1][k])
            x = _col(Xt, j, m)
            d = x @ x                      # <X_j, X_j>
            if d != 0.0:
                da = _step_size(x, e, d)
                if on_step is not None:
                    e_before = e.copy()
                e = _residual_update(e, x, da)
                _coef_update(a, j, da)
                if on_step is not None:
                    on_step(j, e_before, e, da, x @ e_before, d)
            cols += 1
            if refresh_cols and Xt_refresh is not None and cols % refresh_cols == 0:
                e = residual(Xt_refresh, y, m, a)
                res.refreshes += 1
            if (k < n - 1 and check_cols and stop == STOP_REL_RESID
                    and cols % check_cols == 0):
                nrm = float(np.linalg.norm(e))
                if passes(nrm) and (not confirm or confirmed()):
                    res.a, res.e, res.cols, res.sweeps, res.converged = a, e, cols, s - 1, True
                    res.extra["stop_norm"] = nrm
                    return res
        hist.append(float(np.linalg.norm(e)))
        if stop == STOP_REL_GRAD:
            gn = float(np.linalg.norm(gradient(Xt, m, e)))
            res.extra["grad_hist"].append(gn)
            if hist[-1] == 0.0 or gn == 0.0 or gn < tol * res.extra["xty_norm"]:
                res.a, res.e, res.cols, res.sweeps, res.converged = a, e, cols, s, True
                return res
            continue
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


def solve_parallel(Xt, y, m=None, a0=None, max_sweeps=1, thr=1, tol=0.0, stop=STOP_NONE):
    """The parallel solver of Section 7 (Algorithm 2, HPSCDP) in FP64.

    Each sweep first keeps a copy aprev of a.  The columns are then taken in
    consecutive blocks jj = {j, ..., j + thr - 1} (j = 1, thr + 1, ...; the
    last block holds the min(thr, n - j + 1) columns that remain, since the
    printed index set assumes thr divides n).  Every column k of a block
    moves a_k by <X_k, e> / <X_k, X_k> against the SAME residual e (the one
    at the start of the block: the steps of a block are independent and may
    run in parallel); afterwards the residual takes the whole block at once,
    e <- e - X_jj (a_jj - aprev_jj).  thr = 1 is Algorithm 1.  Zero columns
    are skipped as in ``solve``.  Stop rules: STOP_NONE, STOP_REL_CHANGE and
    STOP_REL_RESID at sweep ends, as in ``solve``.

    ``extra["diverged"]`` is True when ||e|| grew over some sweep (Section 7
    reports convergence only for blocks that are small against n: the steps
    of a block ignore one another, so strongly correlated columns in one
    block overshoot).
    """
    n = Xt.shape[0]
    m = Xt.shape[1] if m is None else int(m)
    thr = int(thr)
    if thr < 1:
        raise ValueError("thr must be >= 1")
    y64 = np.asarray(y[:m], dtype=np.float64)
    ynorm = float(np.linalg.norm(y64))
    a = np.zeros(n) if a0 is None else np.array(a0, dtype=np.float64)
    e = y64.copy() if a0 is None else residual(Xt, y, m, a)
    hist = [float(np.linalg.norm(e))]
    d = np.array([_col(Xt, j, m) @ _col(Xt, j, m) for j in range(n)])
    res = OracleResult(a, e, hist, 0, 0, False, int((d == 0.0).sum()))
    res.extra["diverged"] = False
    if stop == STOP_REL_RESID and (hist[0] == 0.0 or hist[0] < tol * ynorm):
        res.converged = True
        return res
    if stop != STOP_NONE and hist[0] == 0.0:
        res.converged = True
        return res
    for s in range(1, max_sweeps + 1):
        aprev = a.copy()
        for j in range(0, n, thr):
            jj = range(j, min(j + thr, n))
            for k in jj:                      # "do in parallel": all read the same e
                if d[k] != 0.0:
                    x = _col(Xt, k, m)
                    a[k] = a[k] + (x @ e) / d[k]
            for k in jj:                      # e <- e - X_jj (a_jj - aprev_jj)
                if a[k] != aprev[k]:
                    e = e - _col(Xt, k, m) * (a[k] - aprev[k])
            res.cols += len(jj)
        hist.append(float(np.linalg.norm(e)))
        if hist[-1] > hist[-2]:
            res.extra["diverged"] = True
        res.sweeps = s
        if not np.isfinite(hist[-1]):
            break
        if stop != STOP_NONE and _sweep_stop(stop, tol, hist, ynorm):
            res.converged = True
            break
    res.a, res.e = a, e
    return res


@dataclass
class SelectResult:
    J: list                       # selected column indices, in selection order
    a: np.ndarray                 # FP64 coefficients (a0 plus the selected steps)
    e: np.ndarray                 # FP64 residual y - X·a
    hist: list                    # ||e||_2 before the first and after each selection
    da: list                      # step taken for each selected column
    scores: list                  # <X_j,e>^2/<X_j,X_j> of each selected column
    stopped: bool = False         # the relative-decrease rule ended the selection


def select_features(Xt, y, m=None, F=1, a0=None, tol=0.0, on_select=None):
    """Feature selection with HPSCD (Section 8, Algorithm 3, HPSCDF) in FP64.

    Start from a = a0 (zero unless given), e = y - X·a, an empty selection J,
    and the column norms <X_j, X_j> (the diagonal of X^T X: the algorithm
    divides element-wise by it).  For f = 1..F:
      * da_j = <X_j, e> / <X_j, X_j> for every column, all against the same
        e (the first step of Algorithm 1's inner loop, for every j at once);
      * E_j = sum_i (e_i - X_ij da_j)^2, the squared error if only column j
        took its step (the printed sum lacks the square and adds a_j; with
        the square and the step alone, E_j is the error the text says is
        minimised: a_j X_j is already out of e);
      * j^ = argmin E_j over the columns not selected yet (J holds F distinct
        features; ties go to the lowest index; zero columns never qualify);
      * J <- (J, j^); a_j^ <- a_j^ + da_j^ (the printed overwrite equals this
        for a column whose coefficient is still zero); e <- e - X_j^ da_j^.
    tol > 0 is the while-loop variant the section describes: the selection
    stops before a column whose step would lower ||e||^2 by less than
    tol * ||e||^2 (the errors stop decreasing).
    on_select(f, E, d): optional hook receiving the vector E of step f.
    """
    n = Xt.shape[0]
    m = Xt.shape[1] if m is None else int(m)
    y64 = np.asarray(y[:m], dtype=np.float64)
    a = np.zeros(n) if a0 is None else np.array(a0, dtype=np.float64)
    e = y64.copy() if a0 is None else residual(Xt, y, m, a)
    d = np.array([_col(Xt, j, m) @ _col(Xt, j, m) for j in range(n)])
    res = SelectResult([], a, e, [float(np.linalg.norm(e))], [], [])
    chosen = np.zeros(n, dtype=bool)
    for f in range(int(F)):
        cand = np.flatnonzero(~chosen & (d != 0.0))
        if cand.size == 0:
            break
        da = np.zeros(n)
        E = np.full(n, np.inf)
        for j in cand:
            x = _col(Xt, j, m)
            da[j] = (x @ e) / d[j]
            E[j] = float(np.sum((e - x * da[j]) ** 2))
        if on_select is not None:
            on_select(f, E, d)
        jh = int(np.argmin(E))           # first index among equal minima
        e2 = float(e @ e)
        if tol > 0.0 and (e2 - E[jh]) < tol * e2:
            res.stopped = True
            break
        res.J.append(jh)
        res.da.append(float(da[jh]))
        res.scores.append(e2 - float(E[jh]))
        chosen[jh] = True
        a[jh] = a[jh] + da[jh]
        e = e - _col(Xt, jh, m) * da[jh]
        res.hist.append(float(np.linalg.norm(e)))
    res.a, res.e = a, e
    return res
