"""Pins of the oracle's variants against facts fixed by the paper and by
mathematics: the gradient stop rule, random column order (Section 2), the
parallel solver (Section 7, Algorithm 2) and feature selection (Section 8,
Algorithm 3).

Each check compares the oracle with a different algorithm, a closed form, a
library routine or brute force, never with a retyped copy of its own step.
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


# ------------------------------------------------------------ gradient stop

def test_rel_grad_stops_where_direct_normal_equation_check_passes():
    """STOP_REL_GRAD stops after the first sweep whose ||X^T(y - X a)|| drops
    below tol·||X^T y||, evaluated here directly from the dense matrix."""
    s = gen.tall_small()
    X = s.X()
    y = s.y.astype(np.float64)
    xty = np.linalg.norm(X.T @ y)
    tol = 1e-7
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, stop=oracle.STOP_REL_GRAD, tol=tol)
    assert r.converged
    ratios = []
    for k in range(1, r.sweeps + 1):
        a = oracle.solve(s.Xt, s.y, s.m, max_sweeps=k).a
        ratios.append(np.linalg.norm(X.T @ (y - X @ a)) / xty)
    assert ratios[-1] < tol
    assert all(q >= tol for q in ratios[:-1])
    assert r.extra["xty_norm"] == pytest.approx(xty, rel=1e-13)
    np.testing.assert_allclose(np.array(r.extra["grad_hist"][1:]) / xty, ratios, rtol=1e-6)


def test_rel_grad_vanishes_at_least_squares_solution():
    """Section 4's limit is the least-squares minimiser, where the normal
    equations hold: the relative gradient falls to rounding level."""
    s = gen.tall_small()
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200, stop=oracle.STOP_REL_GRAD, tol=1e-13)
    assert r.converged and r.sweeps < 200
    X = s.X()
    a_ls = np.linalg.lstsq(X, s.y.astype(np.float64), rcond=None)[0]
    assert np.linalg.norm(r.a - a_ls) / np.linalg.norm(a_ls) < 1e-11


def test_rel_grad_zero_gradient_stops():
    """X^T y = 0 (y orthogonal to every column): a = 0 already solves the
    least-squares problem; the rule stops after one sweep with a unchanged."""
    X = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    y = np.array([0.0, 0.0, 3.0])
    Xt, yy, m = _sys(X, y)
    r = oracle.solve(Xt, yy, m, max_sweeps=10, stop=oracle.STOP_REL_GRAD, tol=1e-3)
    assert r.converged and r.sweeps == 1 and np.all(r.a == 0.0)


# ------------------------------------------------------------- column order

def _gauss_seidel_ordered(X, y, orders):
    """Gauss-Seidel on X^T X a = X^T y visiting the coordinates in the given
    order in every sweep (it never forms the residual e)."""
    A = X.T @ X
    b = X.T @ y
    a = np.zeros(X.shape[1])
    out = []
    for row in orders:
        for j in row:
            a[j] = (b[j] - A[j] @ a + A[j, j] * a[j]) / A[j, j]
        out.append(a.copy())
    return out


def test_identity_order_is_cyclic_bitwise():
    s = gen.tall_small(m=300, n=20)
    ident = np.tile(np.arange(20, dtype=np.int32), (7, 1))
    r0 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=7)
    r1 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=7, order=ident)
    np.testing.assert_array_equal(r0.a, r1.a)
    assert r0.hist == r1.hist


def test_random_order_equals_ordered_gauss_seidel():
    """Any visiting order is coordinate descent on ||y - X a||^2 in that
    order, i.e. Gauss-Seidel on the normal equations in that order."""
    rng = np.random.default_rng(17)
    X = rng.standard_normal((80, 11)) * rng.uniform(0.3, 4, 11)
    y = rng.standard_normal(80)
    orders = gen.column_orders(5, 9, 11)
    gs = _gauss_seidel_ordered(X, y, orders)
    Xt, yy, m = _sys(X, y)
    for s in (1, 2, 5, 9):
        r = oracle.solve(Xt, yy, m, max_sweeps=s, order=orders)
        np.testing.assert_allclose(r.a, gs[s - 1], rtol=1e-11, atol=1e-13)


def test_fixed_permutation_equals_permuted_system():
    """Visiting the columns in a fixed order p equals solving the system with
    columns X[:, p] cyclically, coefficient p[k] taking coefficient k."""
    s = gen.tall_small(m=400, n=15)
    p = np.random.default_rng(3).permutation(15).astype(np.int32)
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=6, order=np.tile(p, (6, 1)))
    rp = oracle.solve(np.ascontiguousarray(s.Xt[p]), s.y, s.m, max_sweeps=6)
    np.testing.assert_array_equal(r.a[p], rp.a)


def test_random_order_converges_to_lstsq_and_is_monotone():
    s = gen.tall_small()
    orders = gen.column_orders(8, 200, s.n)
    r = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200, order=orders)
    a_ls = np.linalg.lstsq(s.X(), s.y.astype(np.float64), rcond=None)[0]
    assert np.linalg.norm(r.a - a_ls) / np.linalg.norm(a_ls) < 1e-12
    h = np.array(r.hist)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-14))


def test_order_must_be_permutations():
    s = gen.tall_small(m=50, n=4)
    with pytest.raises(ValueError):
        oracle.solve(s.Xt, s.y, s.m, max_sweeps=2, order=np.array([[0, 1, 2, 3], [0, 0, 2, 3]]))
    with pytest.raises(ValueError):
        oracle.solve(s.Xt, s.y, s.m, max_sweeps=3, order=np.tile(np.arange(4), (2, 1)))


# ---------------------------------------------------------- parallel solver

def _block_jacobi_gauss_seidel(X, y, thr, sweeps, a0=None):
    """Textbook form of Algorithm 2 on the normal equations A a = b: blocks
    of thr coordinates in order; inside a block every coordinate moves by
    (b_k - A_k a)/A_kk with the SAME a (Jacobi), the block's new values are
    used by later blocks (Gauss-Seidel).  Never forms the residual."""
    A = X.T @ X
    b = X.T @ y
    n = X.shape[1]
    a = np.zeros(n) if a0 is None else np.array(a0, dtype=np.float64)
    out = []
    for _ in range(sweeps):
        for j in range(0, n, thr):
            jj = np.arange(j, min(j + thr, n))
            a[jj] = a[jj] + (b[jj] - A[jj] @ a) / np.diag(A)[jj]
        out.append(a.copy())
    return out


@pytest.mark.parametrize("thr", [1, 3, 4, 7, 16])
def test_parallel_equals_block_jacobi_on_normal_equations(thr):
    rng = np.random.default_rng(23)
    X = rng.standard_normal((120, 16)) * rng.uniform(0.3, 3, 16)
    y = rng.standard_normal(120)
    ref = _block_jacobi_gauss_seidel(X, y, thr, 8)
    Xt, yy, m = _sys(X, y)
    for s in (1, 3, 8):
        r = oracle.solve_parallel(Xt, yy, m, max_sweeps=s, thr=thr)
        np.testing.assert_allclose(r.a, ref[s - 1], rtol=1e-10, atol=1e-12)
        assert r.cols == 16 * s


def test_parallel_thr1_matches_algorithm1_dyadic_exact():
    """thr = 1: Algorithm 2 is Algorithm 1; on the dyadic 2x2 example the
    values are exact: a = (1 + 2^(1-s), 1 - 2^(-s)), e = 2^(-s)(-1, 1)."""
    Xt, y, m = _sys([[1, 1], [0, 1]], [2, 1])
    for s in range(1, 20):
        r = oracle.solve_parallel(Xt, y, m, max_sweeps=s, thr=1)
        assert r.a.tolist() == [1 + 2.0 ** (1 - s), 1 - 2.0 ** (-s)]
        assert r.e.tolist() == [-(2.0 ** -s), 2.0 ** -s]


def test_parallel_thr1_matches_algorithm1():
    s = gen.tall_small(m=500, n=30)
    r1 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=10)
    rp = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=10, thr=1)
    np.testing.assert_allclose(rp.a, r1.a, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(rp.hist, r1.hist, rtol=1e-13)


@pytest.mark.parametrize("thr", [1, 5, 12])
def test_parallel_orthogonal_columns_exact_after_one_sweep(thr):
    """Orthogonal columns do not interact: one sweep gives the least-squares
    solution for every block size."""
    s = gen.orthogonal_columns(200, 12, seed=5)
    r = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=1, thr=thr)
    a_ls = np.linalg.lstsq(s.X(), s.y, rcond=None)[0]
    np.testing.assert_allclose(r.a, a_ls, rtol=1e-10)


def test_parallel_last_block_is_short():
    """n = 10, thr = 4: blocks {0..3}, {4..7}, {8, 9} (the last block takes
    the columns that remain)."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((60, 10))
    y = rng.standard_normal(60)
    ref = _block_jacobi_gauss_seidel(X, y, 4, 3)
    Xt, yy, m = _sys(X, y)
    r = oracle.solve_parallel(Xt, yy, m, max_sweeps=3, thr=4)
    np.testing.assert_allclose(r.a, ref[-1], rtol=1e-10, atol=1e-12)
    assert r.cols == 30


def test_parallel_correlated_block_diverges_small_block_converges():
    """Three nearly equal columns in one block: each takes the full step
    against the same residual, together three times the fit, so ||e|| grows
    (the Jacobi factor 1 - 3 has modulus above one: the divergence Section 7
    warns of for blocks that are not small).  Apart (thr = 1) the method
    converges monotonically."""
    s = gen.correlated_group(400, 8, seed=4, k=3, eps=1e-3, at=0, dtype=np.float64)
    bad = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=30, thr=4)
    assert bad.extra["diverged"]
    assert bad.hist[-1] > bad.hist[0]
    good = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=30, thr=1)
    assert not good.extra["diverged"]
    h = np.array(good.hist)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-14))


def test_parallel_small_thr_converges_to_lstsq():
    """Section 7: with thr small against n (here n/10) the method converges;
    on the 2000x50 Gaussian system it reaches the least-squares solution."""
    s = gen.tall_small()
    r = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=300, thr=5)
    a_ls = np.linalg.lstsq(s.X(), s.y.astype(np.float64), rcond=None)[0]
    assert np.linalg.norm(r.a - a_ls) / np.linalg.norm(a_ls) < 1e-10
    assert not r.extra["diverged"]


def test_parallel_stop_rules():
    s = gen.tall_small(m=800, n=40)
    r = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=200, thr=4,
                              stop=oracle.STOP_REL_CHANGE, tol=1e-6)
    assert r.converged
    h = r.hist
    assert (h[-2] - h[-1]) < 1e-6 * h[-1]
    assert all((h[k - 1] - h[k]) >= 1e-6 * h[k] for k in range(1, len(h) - 1))


# --------------------------------------------------------- feature selection

def test_select_error_is_pythagorean_split():
    """E_j = ||e - X_j da_j||^2 = ||e||^2 - <X_j,e>^2/<X_j,X_j> (the step
    leaves e - X_j da_j orthogonal to X_j, Section 4)."""
    s = gen.tall_small(m=300, n=25)
    X = s.X()
    seen = []

    def hook(f, E, d):
        seen.append(E.copy())

    r = oracle.select_features(s.Xt, s.y, s.m, F=6, on_select=hook)
    e = s.y.astype(np.float64)
    for f, E in enumerate(seen):
        g = X.T @ e
        closed = e @ e - g * g / (X * X).sum(0)
        cand = np.isfinite(E)
        np.testing.assert_allclose(E[cand], closed[cand], rtol=1e-9, atol=1e-9 * (e @ e))
        jh = r.J[f]
        e = e - X[:, jh] * (g[jh] / (X[:, jh] @ X[:, jh]))


def test_select_matches_brute_force_one_column_lstsq():
    """Brute force: at every step the selected column is the one whose
    one-column least-squares fit of the current residual (numpy.linalg.lstsq)
    leaves the smallest residual, among columns not yet selected."""
    s = gen.tall_small(m=200, n=30)
    X = s.X()
    r = oracle.select_features(s.Xt, s.y, s.m, F=10)
    e = s.y.astype(np.float64)
    used = set()
    for f in range(10):
        best, bj, bc = np.inf, -1, 0.0
        for j in range(30):
            if j in used:
                continue
            c, res, *_ = np.linalg.lstsq(X[:, [j]], e, rcond=None)
            rr = float(res[0]) if res.size else float(np.sum((e - X[:, j] * c[0]) ** 2))
            if rr < best:
                best, bj, bc = rr, j, float(c[0])
        assert r.J[f] == bj
        assert r.da[f] == pytest.approx(bc, rel=1e-10)
        used.add(bj)
        e = e - X[:, bj] * bc
        assert r.hist[f + 1] == pytest.approx(math.sqrt(best), rel=1e-9)


def test_select_orthogonal_columns_all_is_lstsq():
    """Orthogonal columns: selection order is by decreasing
    <X_j,y>^2/<X_j,X_j>, and selecting all n gives the least-squares a."""
    s = gen.orthogonal_columns(150, 10, seed=9)
    X = s.X()
    r = oracle.select_features(s.Xt, s.y, s.m, F=10)
    score = (X.T @ s.y) ** 2 / (X * X).sum(0)
    assert r.J == list(np.argsort(-score, kind="stable"))
    a_ls = np.linalg.lstsq(X, s.y, rcond=None)[0]
    np.testing.assert_allclose(r.a, a_ls, rtol=1e-10, atol=1e-12)


def test_select_recovers_planted_support():
    """y = 5 X_3 - 4 X_11 + 3 X_20 (plus small noise) over Gaussian columns:
    the first three selections are the planted columns."""
    rng = np.random.default_rng(31)
    X = rng.standard_normal((500, 40))
    y = 5 * X[:, 3] - 4 * X[:, 11] + 3 * X[:, 20] + 0.01 * rng.standard_normal(500)
    Xt, yy, m = _sys(X, y)
    r = oracle.select_features(Xt, yy, m, F=3)
    assert sorted(r.J) == [3, 11, 20]
    np.testing.assert_allclose(r.a[[3, 11, 20]], [5, -4, 3], rtol=0.05)


def test_select_distinct_skips_zero_columns_and_stops():
    s = gen.tall_small(m=100, n=12)
    Xt = s.Xt.astype(np.float64).copy()
    Xt[5, :] = 0.0
    r = oracle.select_features(Xt, s.y, s.m, F=20)
    assert len(r.J) == 11 and len(set(r.J)) == 11 and 5 not in r.J
    h = np.array(r.hist)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-14))
    # while-loop variant: stop before a step that lowers ||e||^2 by less
    # than tol·||e||^2
    tol = 0.02
    rt = oracle.select_features(Xt, s.y, s.m, F=20, tol=tol)
    assert rt.stopped and rt.J == r.J[: len(rt.J)]
    dec = [(h[k] ** 2 - h[k + 1] ** 2) / h[k] ** 2 for k in range(len(h) - 1)]
    k = len(rt.J)
    assert all(q >= tol for q in dec[:k]) and dec[k] < tol


def test_select_with_initial_guess():
    """a0 = a_true on a consistent system: e = y - X a0 = 0, every step is
    zero; the selection keeps a = a0."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((50, 6))
    a0 = rng.standard_normal(6)
    Xt, yy, m = _sys(X, X @ a0)
    r = oracle.select_features(Xt, yy, m, F=3, a0=a0)
    np.testing.assert_allclose(r.a, a0, atol=1e-13)
    assert r.hist[0] < 1e-12


# --------------------------------------------------------- planted mistakes

def _bad_index_col(Xt, j, m):
    return np.asarray(Xt[(j + 1) % Xt.shape[0], :m], dtype=np.float64)


@pytest.mark.parametrize("where", ["parallel", "select"])
def test_variant_pins_catch_planted_column_mistake(where, monkeypatch):
    """Plant a wrong column index in the oracle's column access and check
    that the pins above reject it."""
    monkeypatch.setattr(ho, "_col", _bad_index_col)
    with pytest.raises(AssertionError):
        if where == "parallel":
            test_parallel_equals_block_jacobi_on_normal_equations(3)
        else:
            test_select_matches_brute_force_one_column_lstsq()
