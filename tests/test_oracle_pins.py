"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's own step: each compares it with a
closed form, a different algorithm, a library routine or an invariant proved
in the paper (Section 4), so that a dropped term, a wrong sign, a wrong index
or a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import hpscd_oracle as ho
from workloads import gen


def _sys(X, y):
    X = np.asarray(X, dtype=np.float64)
    return np.ascontiguousarray(X.T), np.asarray(y, dtype=np.float64), X.shape[0]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dyadic_2x2_closed_form(dtype):
    """X = [[1,1],[0,1]], y = (2,1), a0 = 0.  Working Algorithm 1 by hand gives,
    after s >= 1 sweeps, a = (1 + 2^(1-s), 1 - 2^(-s)) and
    e = 2^(-s)·(-1, 1); every value is dyadic, so equality is exact."""
    Xt, y, m = _sys([[1, 1], [0, 1]], [2, 1])
    Xt = Xt.astype(dtype)
    for s in range(1, 24):
        r = oracle.solve(Xt, y.astype(dtype), m, max_sweeps=s)
        assert r.a.tolist() == [1 + 2.0 ** (1 - s), 1 - 2.0 ** (-s)]
        assert r.e.tolist() == [-(2.0 ** -s), 2.0 ** -s]
        assert r.hist[-1] == math.sqrt(2.0) * 2.0 ** -s
        assert r.sweeps == s and r.cols == 2 * s


def test_single_column_closed_form():
    """n = 1: one step is the one-variable least-squares fit
    a = <x, y>/<x, x> (Section 3, the step-size derivation)."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(300)
    y = rng.standard_normal(300)
    Xt, y, m = _sys(x[:, None], y)
    r = oracle.solve(Xt, y, m, max_sweeps=1)
    assert r.a[0] == pytest.approx(float(np.dot(x, y) / np.dot(x, x)), rel=1e-14)
    r3 = oracle.solve(Xt, y, m, max_sweeps=3)
    assert r3.a[0] == pytest.approx(r.a[0], rel=1e-14)


def test_orthogonal_columns_exact_after_one_sweep():
    """Mutually orthogonal columns: each step removes exactly the projection
    on X_j, so one sweep yields a_j = <X_j,y>/<X_j,X_j> and the least-squares
    residual of numpy.linalg.lstsq."""
    s = gen.orthogonal_columns(200, 12, seed=5)
    X = s.X()
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=1)
    expect = (X.T @ s.y) / (X * X).sum(0)
    np.testing.assert_allclose(r.a, expect, rtol=1e-12)
    a_ls = np.linalg.lstsq(X, s.y, rcond=None)[0]
    np.testing.assert_allclose(r.a, a_ls, rtol=1e-10)
    np.testing.assert_allclose(r.e, s.y - X @ a_ls, atol=1e-12)


def test_diagonal_square_system():
    """Diagonal square X: a_j = y_j / X_jj after one sweep, residual zero."""
    d = np.array([2.0, -0.5, 4.0, 1.0, 8.0])
    y = np.array([1.0, 2.0, -3.0, 0.25, 1.5])
    Xt, y, m = _sys(np.diag(d), y)
    r = oracle.solve(Xt, y, m, max_sweeps=1)
    np.testing.assert_array_equal(r.a, y / d)
    assert np.all(r.e == 0.0)


# ------------------------------------------------ different algorithm / library

def _gauss_seidel_normal_equations(X, y, sweeps):
    """Textbook Gauss-Seidel on X^T X a = X^T y (ascending j, latest values).
    Independent of the oracle: it never forms the residual e."""
    A = X.T @ X
    b = X.T @ y
    a = np.zeros(X.shape[1])
    out = []
    for _ in range(sweeps):
        for j in range(len(a)):
            a[j] = (b[j] - A[j] @ a + A[j, j] * a[j]) / A[j, j]
        out.append(a.copy())
    return out


def test_iterates_equal_gauss_seidel_on_normal_equations():
    """In exact arithmetic Algorithm 1 is Gauss-Seidel on the normal
    equations; the iterates agree sweep by sweep up to rounding."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((60, 9)) * rng.uniform(0.2, 5, 9)
    y = rng.standard_normal(60)
    gs = _gauss_seidel_normal_equations(X, y, 12)
    Xt, yy, m = _sys(X, y)
    for s in range(1, 13):
        r = oracle.solve(Xt, yy, m, max_sweeps=s)
        np.testing.assert_allclose(r.a, gs[s - 1], rtol=1e-11, atol=1e-13)


def test_tall_small_converges_to_lstsq():
    """Section 4 limit: the iteration reaches the least-squares minimiser.
    On the 2000x50 Gaussian system, 200 sweeps agree with numpy.linalg.lstsq
    to 1e-12 relative, and the residual equals e_min."""
    s = gen.tall_small()
    X = s.X()
    y = s.y.astype(np.float64)
    a_ls, res_ls, *_ = np.linalg.lstsq(X, y, rcond=None)
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200)
    assert np.linalg.norm(r.a - a_ls) / np.linalg.norm(a_ls) < 1e-12
    assert r.hist[-1] ** 2 == pytest.approx(float(res_ls[0]), rel=1e-10)
    # the error after 5 sweeps is much larger than after 20 (geometric rate)
    e5 = np.linalg.norm(oracle.solve(s.Xt, s.y, s.m, max_sweeps=5).a - a_ls)
    e20 = np.linalg.norm(oracle.solve(s.Xt, s.y, s.m, max_sweeps=20).a - a_ls)
    assert e20 < 1e-6 * e5


@pytest.mark.parametrize("kind,sweeps", [("perturbed_identity", 80), ("orth_scaled", 1)])
def test_exact_recovery_square_consistent(kind, sweeps):
    """Consistent, well-conditioned square systems: e_min = 0 and the method
    recovers a_true (Section 4, minimum-error definition)."""
    s = gen.square_well_conditioned(64, seed=3, kind=kind)
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=sweeps)
    assert np.linalg.norm(r.a - s.a_true) / np.linalg.norm(s.a_true) < 1e-12
    assert r.hist[-1] < 1e-12 * np.linalg.norm(s.y)


def test_wide_consistent_residual_vanishes():
    """Wide full-row-rank system: a is not unique but the limit residual is
    y - P_range(X) y = 0.  Compare e with the lstsq residual."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((30, 90))
    y = rng.standard_normal(30)
    Xt, yy, m = _sys(X, y)
    r = oracle.solve(Xt, yy, m, max_sweeps=300)
    assert np.linalg.norm(r.e) < 1e-12 * np.linalg.norm(y)
    np.testing.assert_allclose(X @ r.a, y, atol=1e-11)


def test_rank_deficient_tall_residual_is_projection():
    """Duplicate columns: a is not unique, the residual limit is the lstsq one."""
    rng = np.random.default_rng(4)
    B = rng.standard_normal((80, 5))
    X = np.concatenate([B, B[:, :2] * 2.0], axis=1)
    y = rng.standard_normal(80)
    Xt, yy, m = _sys(X, y)
    r = oracle.solve(Xt, yy, m, max_sweeps=400)
    a_ls = np.linalg.lstsq(X, y, rcond=None)[0]
    np.testing.assert_allclose(r.e, y - X @ a_ls, atol=1e-11)


# ------------------------------------------------ invariants of Section 4

def test_step_invariants_section4():
    """After every step: X_j^T e_{k+1} = 0 (orthogonality), the Pythagorean
    split ||e_k||^2 = da^2 ||X_j||^2 + ||e_{k+1}||^2, monotone decrease, and
    e stays equal to y - X·a."""
    rng = np.random.default_rng(9)
    m, n = 120, 15
    X = rng.standard_normal((m, n)) * rng.uniform(0.1, 10.0, n)
    y = rng.standard_normal(m)
    Xt, yy, _ = _sys(X, y)
    u = np.finfo(np.float64).eps
    seen = []

    def hook(j, eb, ea, da, g, d):
        xj = X[:, j]
        ne_b = np.linalg.norm(eb)
        assert abs(xj @ ea) <= 50 * math.sqrt(m) * u * np.linalg.norm(xj) * ne_b
        assert ne_b ** 2 == pytest.approx(da * da * d + ea @ ea, rel=1e-12, abs=1e-14 * ne_b ** 2)
        assert g * g / d == pytest.approx(ne_b ** 2 - ea @ ea, rel=1e-6, abs=1e-12 * ne_b ** 2)
        assert ea @ ea <= (eb @ eb) * (1 + 4 * u * math.sqrt(m)) + 1e-300
        seen.append(j)

    r = oracle.solve(Xt, yy, m, max_sweeps=6, on_step=hook)
    assert seen == list(range(n)) * 6
    np.testing.assert_allclose(r.e, y - X @ r.a, atol=1e-12 * np.linalg.norm(y))
    h = np.array(r.hist)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-15))


def test_column_power_of_two_scaling_symmetry():
    """Scaling X_j by 2^k leaves every e bitwise unchanged and divides a_j by
    2^k (da scales by 2^-k, X_j·da does not change)."""
    s = gen.tall_small(m=300, n=20)
    Xt2 = s.Xt.astype(np.float64).copy()
    scale = np.array([2.0 ** k for k in rng_ints(20)])
    Xt2 *= scale[:, None]
    r1 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=7)
    r2 = oracle.solve(Xt2, s.y, s.m, max_sweeps=7)
    np.testing.assert_array_equal(r1.e, r2.e)
    np.testing.assert_array_equal(r1.a, r2.a * scale)


def rng_ints(n):
    return np.random.default_rng(0).integers(-6, 7, n)


def test_column_permutation_same_limit():
    """Full-rank tall systems reach the same limit in any column order."""
    s = gen.tall_small(m=400, n=12)
    perm = np.random.default_rng(1).permutation(12)
    r1 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200)
    r2 = oracle.solve(s.Xt[perm], s.y, s.m, max_sweeps=200)
    np.testing.assert_allclose(r2.a, r1.a[perm], rtol=1e-12, atol=1e-14)


def test_zero_column_is_skipped():
    """Reading: a zero column contributes nothing and is counted."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 6))
    X[:, 2] = 0.0
    y = rng.standard_normal(50)
    Xt, yy, m = _sys(X, y)
    r = oracle.solve(Xt, yy, m, max_sweeps=100)
    assert r.zero_cols == 1 and r.a[2] == 0.0
    keep = [0, 1, 3, 4, 5]
    a_ls = np.linalg.lstsq(X[:, keep], y, rcond=None)[0]
    np.testing.assert_allclose(r.a[keep], a_ls, rtol=1e-10)
    z = oracle.solve(np.zeros((3, 50)), yy, m, max_sweeps=3)
    assert z.zero_cols == 3 and np.all(z.a == 0) and np.array_equal(z.e, y)


def test_warm_start_and_resume():
    """a0 = the result of k sweeps, resumed for k more, equals 2k sweeps
    (the initial guess of Algorithm 1 and e = y - X·a0)."""
    s = gen.tall_small(m=500, n=30)
    r4 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=4)
    r2 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=2)
    rr = oracle.solve(s.Xt, s.y, s.m, a0=r2.a, max_sweeps=2)
    np.testing.assert_allclose(rr.a, r4.a, rtol=1e-12)
    assert rr.hist[0] == pytest.approx(r2.hist[-1], rel=1e-12)


# ------------------------------------------------ stopping readings

def test_stop_rel_change():
    s = gen.tall_small()
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200, tol=1e-6, stop=oracle.STOP_REL_CHANGE)
    assert r.converged and r.sweeps < 200
    h = r.hist
    assert (h[-2] - h[-1]) < 1e-6 * h[-1]
    assert all((h[k - 1] - h[k]) >= 1e-6 * h[k] for k in range(1, len(h) - 1))


def test_stop_rel_resid_sweep_and_column_checks():
    s = gen.square_well_conditioned(64, seed=8)
    ny = np.linalg.norm(s.y)
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=500, tol=1e-9, stop=oracle.STOP_REL_RESID)
    assert r.converged and r.hist[-1] < 1e-9 * ny and r.hist[-2] >= 1e-9 * ny
    rc = oracle.solve(s.Xt, s.y, s.m, max_sweeps=500, tol=1e-9,
                      stop=oracle.STOP_REL_RESID, check_cols=8)
    assert rc.converged and rc.cols % 8 == 0 and rc.cols <= r.cols
    assert rc.extra.get("stop_norm", rc.hist[-1]) < 1e-9 * ny
    # already converged before the first sweep: zero sweeps
    r0 = oracle.solve(s.Xt, s.y, s.m, a0=s.a_true, max_sweeps=5, tol=1e-9,
                      stop=oracle.STOP_REL_RESID)
    assert r0.converged and r0.sweeps == 0


# ------------------------------------------------ bfloat16 storage form

def test_bf16_round_matches_torch():
    """Round-to-nearest-even to bfloat16 agrees with torch's conversion."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(10000).astype(np.float32),
        (rng.standard_normal(1000) * 1e-39).astype(np.float32),   # subnormals
        (rng.standard_normal(1000) * 1e37).astype(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.4e38, -3.4e38], np.float32),
    ])
    u = x.view(np.uint32)
    ties = ((u & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)  # exact halfway
    x = np.concatenate([x, ties[:2000]])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = ho.bf16_round(x)
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(ho.bf16_round(np.array([np.nan], np.float32)))[0]


def test_bf16_form_reduces_to_plain_when_exact():
    """If X is already bfloat16-representable, the storage form is Algorithm 1
    (the refreshes recompute the same e up to rounding)."""
    s = gen.tall_small(m=256, n=16)
    Xb = ho.bf16_round(s.Xt)
    r1 = oracle.solve(Xb, s.y, s.m, max_sweeps=10)
    r2 = oracle.solve_bf16_refresh(Xb, s.y, s.m, max_sweeps=10, refresh_cols=16)
    np.testing.assert_allclose(r2.a, r1.a, rtol=1e-11)
    assert r2.refreshes == 10


def test_bf16_form_refresh_restores_accuracy():
    """Without refresh the true residual (against FP32 X) stalls near the
    bfloat16 floor; refreshing e from FP32 X drives it well below."""
    s = gen.wide(m=200, n=2000, seed=5)
    X32 = s.Xt
    r_no = oracle.solve_bf16_refresh(X32, s.y, s.m, max_sweeps=40)
    r_yes = oracle.solve_bf16_refresh(X32, s.y, s.m, max_sweeps=40, refresh_cols=2000)
    f_no = oracle.final_rel_resid(X32, s.y, s.m, r_no.a)
    f_yes = oracle.final_rel_resid(X32, s.y, s.m, r_yes.a)
    assert 1e-4 < f_no < 1e-1
    assert f_yes < 1e-3 * f_no
    # right after a refresh the running residual is the exact one
    np.testing.assert_allclose(r_yes.e, oracle.residual(X32, s.y, s.m, r_yes.a), atol=1e-12)


def test_bf16_relative_residual_stop_is_confirmed():
    """The relative-residual rule is a statement about the true residual
    y - X·a.  In the storage form the running residual drifts from it (below
    the bfloat16 floor it is meaningless), so a stop it signals must be
    confirmed on the recomputed residual: every converged result then has a
    true relative residual under tol, which the unconfirmed rule misses."""
    s = gen.wide(m=200, n=2000, seed=5)
    X32, tol = s.Xt, 1e-5
    kw = dict(max_sweeps=60, stop=oracle.STOP_REL_RESID, tol=tol, check_cols=100)
    bad = oracle.solve(ho.bf16_round(X32), s.y, s.m, **kw)          # running residual only
    assert bad.converged and oracle.final_rel_resid(X32, s.y, s.m, bad.a) > 1e-4
    r = oracle.solve_bf16_refresh(X32, s.y, s.m, refresh_cols=1000, **kw)
    assert r.converged
    assert oracle.final_rel_resid(X32, s.y, s.m, r.a) < tol
    assert r.cols % 100 == 0 and r.refreshes >= r.cols // 1000 + 1


def test_batch_equals_single():
    b = gen.batch(seed=4, count=6, m_lo=64, m_hi=300, n_lo=3, n_hi=20)
    rs = oracle.solve_batch(b, max_sweeps=5)
    for i, r in enumerate(rs):
        s = b.system(i)
        r1 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=5)
        np.testing.assert_array_equal(r.a, r1.a)


def test_batch_warm_start_pool():
    """a0pool: each system starts from its own slice of the pool (at its
    a_off), and the result equals the single solve started from that slice,
    which in turn continues the zero-start iteration exactly: k sweeps from
    the iterate after j sweeps equal j + k sweeps from zero (up to rounding
    of the recomputed starting residual)."""
    b = gen.batch(seed=4, count=5, m_lo=64, m_hi=300, n_lo=3, n_hi=20)
    first = oracle.solve_batch(b, max_sweeps=3)
    a0pool = np.zeros(b.a_size)
    for i, r in enumerate(first):
        ao = int(b.table[i, 5])
        a0pool[ao: ao + len(r.a)] = r.a
    warm = oracle.solve_batch(b, a0pool=a0pool, max_sweeps=4)
    for i, r in enumerate(warm):
        s = b.system(i)
        full = oracle.solve(s.Xt, s.y, s.m, max_sweeps=7)
        np.testing.assert_allclose(r.a, full.a, rtol=1e-9, atol=1e-12)
        ao = int(b.table[i, 5])
        r1 = oracle.solve(s.Xt, s.y, s.m, a0=a0pool[ao: ao + s.n], max_sweeps=4)
        np.testing.assert_array_equal(r.a, r1.a)


# ------------------------------------------------ planted mistakes

def _run_pins():
    """The pins of Algorithm 1 above; returns the names of those that fail."""
    pins = [
        lambda: test_dyadic_2x2_closed_form(np.float64),
        test_single_column_closed_form,
        test_orthogonal_columns_exact_after_one_sweep,
        test_diagonal_square_system,
        test_iterates_equal_gauss_seidel_on_normal_equations,
        test_step_invariants_section4,
    ]
    failed = []
    for p in pins:
        try:
            p()
        except Exception as exc:  # a wrong oracle may also fail by raising
            failed.append((getattr(p, "__name__", "dyadic"), type(exc).__name__))
    return failed


def test_pins_pass_on_the_oracle():
    assert _run_pins() == []


@pytest.mark.parametrize("mutant", ["sign", "index", "transpose", "drop_norm", "stale_residual"])
def test_pins_catch_planted_mistakes(mutant, monkeypatch):
    """Plant a plausible mistake IN the oracle (each line of Algorithm 1's
    inner loop is a function of the oracle module that is replaced here, on
    the CPU) and check that the pins above reject it."""
    orig_col = ho._col
    if mutant == "sign":         # e <- e + X_j da
        monkeypatch.setattr(ho, "_residual_update", lambda e, x, da: e + x * da)
    elif mutant == "index":      # a_{j+1} <- a_{j+1} + da
        def coef(a, j, da):
            a[(j + 1) % len(a)] += da
        monkeypatch.setattr(ho, "_coef_update", coef)
    elif mutant == "transpose":  # rows of X taken for its columns
        def col_t(Xt, j, m):
            return np.asarray(Xt[:m, j] if Xt.shape[0] >= m else orig_col(Xt, j, m), dtype=np.float64)
        monkeypatch.setattr(ho, "_col", col_t)
    elif mutant == "drop_norm":  # da = <X_j, e> without the division
        monkeypatch.setattr(ho, "_step_size", lambda x, e, d: x @ e)
    else:                        # the residual never updated
        monkeypatch.setattr(ho, "_residual_update", lambda e, x, da: e)
    assert _run_pins(), f"no pin rejects the '{mutant}' mistake"
