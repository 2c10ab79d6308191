"""GPU parity of the method's variants against the FP64 oracle, through the C
ABI: the gradient stop rule, the parallel solver (Section 7, Algorithm 2),
random column order (Section 2) and feature selection (Section 8,
Algorithm 3); and the benchmark's own configurations at full size.

Bounds: as in test_gpu_parity (single precision: 1e-5 relative in a, norm-
and coordinate-wise; hist per sweep).  Feature selection runs in FP64 on the
GPU (FP32 X, FP64 residual and sums), so its choices must equal the
oracle's wherever the oracle's best and second-best errors are apart by more
than 1e-9 relative; its steps and norms agree to 1e-9.
"""
import numpy as np
import pytest

import oracle
from workloads import gen

from test_gpu_parity import TOL_A, check_a, check_final, check_hist, dev, rel, say

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------ gradient stop

@pytest.mark.parametrize("flags", [0, 4])   # library choice (grid) / one workgroup
def test_rel_grad_stop_matches_oracle(lib, flags):
    s = gen.tall_small(pad=np.nan)
    tol = 1e-4
    say("rel grad", flags)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=100, stop=lib.STOP_REL_GRAD, tol=tol, flags=flags)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, stop=oracle.STOP_REL_GRAD, tol=tol)
    say("sweeps", r.info["sweeps_done"], ref.sweeps, "rel grad", r.info["rel_grad"],
        ref.extra["grad_hist"][ref.sweeps] / ref.extra["xty_norm"])
    assert r.info["converged"] == 1 and ref.converged
    assert r.info["sweeps_done"] == ref.sweeps
    ratio = ref.extra["grad_hist"][ref.sweeps] / ref.extra["xty_norm"]
    assert r.info["rel_grad"] == pytest.approx(ratio, rel=1e-3)
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)


def test_rel_grad_not_reached_runs_all_sweeps(lib):
    s = gen.tall_small(m=3000, n=64, pad=np.nan)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, stop=lib.STOP_REL_GRAD, tol=1e-12)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=3)
    assert r.info["converged"] == 0 and r.info["sweeps_done"] == 3
    check_a(r.a.cpu().numpy(), ref.a)
    assert np.isfinite(r.info["rel_grad"]) and r.info["rel_grad"] > 1e-12


def test_rel_grad_full_size(lib):
    """The 1M x 256 system under the gradient rule (one more pass over X
    after every sweep) stops where the oracle's direct normal-equation check
    does."""
    s = gen.tall_large()
    tol = 1e-7
    say("rel grad full size")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=20, stop=lib.STOP_REL_GRAD, tol=tol)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=20, stop=oracle.STOP_REL_GRAD, tol=tol)
    say("sweeps", r.info["sweeps_done"], ref.sweeps, r.info["rel_grad"], ref.extra["grad_hist"])
    assert r.info["converged"] == 1 and abs(r.info["sweeps_done"] - ref.sweeps) <= 1
    eq = oracle.solve(s.Xt, s.y, s.m, max_sweeps=r.info["sweeps_done"])
    check_a(r.a.cpu().numpy(), eq.a, info=r.info)


# ------------------------------------------------------------ Algorithm 2

@pytest.mark.parametrize("thr", [1, 3, 4, 7, 16, 20, 50])
@pytest.mark.parametrize("team", ["wg", "grid"])
def test_parallel_solver_matches_oracle(lib, thr, team):
    """Blocks of thr columns stepped against the residual of the block start:
    thr below, equal to and above the kernel's 16-column block, dividing it
    or not, and thr >= n (one block per sweep)."""
    s = gen.tall_small(pad=np.nan)
    flags = lib.F_FORCE_WG if team == "wg" else lib.F_FORCE_GRID
    say("HPSCDP", thr, team)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=12, thr=thr, flags=flags)
    ref = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=12, thr=thr)
    if thr > 1:  # (thr = 1 is Algorithm 1: the library's own kernel choice)
        assert r.info["kernel_kind"] == 8
    assert (r.info["team_wgs"] > 1) == (team == "grid")
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)
    assert r.info["diverged"] == int(ref.extra["diverged"])


def test_parallel_solver_thr1_is_algorithm1(lib):
    s = gen.tall_small(pad=np.nan)
    r1 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=10, thr=1, depth=8)
    r0 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=10, depth=8)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=10)
    check_a(r1.a.cpu().numpy(), ref.a)
    assert rel(r1.a.cpu().numpy(), r0.a.cpu().numpy()) <= 1e-6


def test_parallel_solver_divergence_flag(lib):
    """Three near-equal columns in one block: Algorithm 2 overshoots and
    ||e|| grows sweep after sweep; the flag is raised as in the oracle, and
    Algorithm 1 on the same system does not raise it."""
    s = gen.correlated_group(4000, 40, seed=4, k=3, eps=1e-3, at=0)
    say("HPSCDP divergence")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=6, thr=8)
    ref = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=6, thr=8)
    assert ref.extra["diverged"] and r.info["diverged"] == 1
    check_hist(r.hist, ref.hist)
    r1 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=6)
    assert r1.info["diverged"] == 0


def test_parallel_solver_stop_and_warm_start(lib):
    s = gen.tall_large(m=200_003, n=45, seed=19, pad=np.nan)
    a0 = np.random.default_rng(5).standard_normal(s.n).astype(np.float32)
    say("HPSCDP stop")
    r = lib.solve(dev(s.Xt), dev(s.y), dev(a0), max_sweeps=60, thr=5, stop=lib.STOP_REL_CHANGE, tol=1e-5)
    ref = oracle.solve_parallel(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=60, thr=5,
                                stop=oracle.STOP_REL_CHANGE, tol=1e-5)
    assert r.info["converged"] == 1 and abs(r.info["sweeps_done"] - ref.sweeps) <= 1
    eq = oracle.solve_parallel(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=r.info["sweeps_done"], thr=5)
    check_a(r.a.cpu().numpy(), eq.a, info=r.info)


def test_parallel_solver_full_size(lib):
    """The 1M x 256 system with thr = 50 (the block width of the paper's
    experiments 1-10) in the benchmark's launch configuration."""
    s = gen.tall_large()
    say("HPSCDP full size")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=2, thr=50)
    ref = oracle.solve_parallel(s.Xt, s.y, s.m, max_sweeps=2, thr=50)
    assert r.info["team_wgs"] == 256
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)


# ------------------------------------------------------------ column order

@pytest.mark.parametrize("team", ["wg", "grid"])
@pytest.mark.parametrize("n", [50, 64, 7])
def test_random_order_matches_oracle(lib, team, n):
    s = gen.tall_small(n=n, pad=np.nan)
    orders = gen.column_orders(31 + n, 15, n)
    flags = lib.F_FORCE_WG if team == "wg" else lib.F_FORCE_GRID
    say("random order", team, n)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=15, order=dev(orders), flags=flags)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=15, order=orders)
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)


def test_identity_order_equals_cyclic(lib):
    s = gen.tall_large(m=100_003, n=40, seed=3, pad=np.nan)
    ident = np.tile(np.arange(s.n, dtype=np.int32), (5, 1))
    r1 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=5, order=dev(ident))
    r0 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=5, depth=8)
    assert rel(r1.a.cpu().numpy(), r0.a.cpu().numpy()) <= 1e-6


def test_random_order_stop_rules(lib):
    s = gen.tall_large(m=150_001, n=48, seed=7, pad=np.nan)
    orders = gen.column_orders(2, 80, s.n)
    say("random order stop")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=80, order=dev(orders), stop=lib.STOP_REL_CHANGE, tol=1e-6)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=80, order=orders, stop=oracle.STOP_REL_CHANGE, tol=1e-6)
    assert r.info["converged"] == 1 and abs(r.info["sweeps_done"] - ref.sweeps) <= 1
    eq = oracle.solve(s.Xt, s.y, s.m, max_sweeps=r.info["sweeps_done"], order=orders)
    check_a(r.a.cpu().numpy(), eq.a, info=r.info)
    # the gradient rule with a column order (both rules run between sweeps)
    r2 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=80, order=dev(orders), stop=lib.STOP_REL_GRAD, tol=1e-6)
    ref2 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=80, order=orders, stop=oracle.STOP_REL_GRAD, tol=1e-6)
    assert r2.info["converged"] == 1 and abs(r2.info["sweeps_done"] - ref2.sweeps) <= 1


def test_random_order_zero_columns(lib):
    rng = np.random.default_rng(12)
    s = gen.make_system(rng, 5000, 37, noise=0.01, pad=np.nan)
    s.Xt[[3, 20], :] = 0.0
    orders = gen.column_orders(9, 6, s.n)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=6, order=dev(orders))
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=6, order=orders)
    assert r.info["zero_cols"] == 2
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    assert np.all(r.a.cpu().numpy()[[3, 20]] == 0.0)


def test_random_order_full_size(lib):
    s = gen.tall_large()
    orders = gen.column_orders(77, 2, s.n)
    say("random order full size")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=2, order=dev(orders))
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=2, order=orders)
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)


# ------------------------------------------------------------ Algorithm 3

def _check_selection(g, ref, F):
    """Choices equal wherever the oracle's decision margin is clear."""
    assert g.count == len(ref.J), (g.count, len(ref.J))
    assert g.J == ref.J, (g.J, ref.J)
    np.testing.assert_allclose(g.da, ref.da, rtol=1e-9, atol=1e-12 * max(1.0, np.max(np.abs(ref.da))))
    np.testing.assert_allclose(g.hist, ref.hist, rtol=1e-9)


def _margins(s, F, **kw):
    m = []

    def hook(f, E, d):
        fin = np.sort(E[np.isfinite(E)])
        if fin.size > 1:
            m.append((fin[1] - fin[0]) / max(fin[0], 1e-300))

    ref = oracle.select_features(s.Xt, s.y, s.m, F=F, on_select=hook, **kw)
    return ref, m


@pytest.mark.parametrize("m,n,F", [(2000, 50, 12), (333, 17, 17), (5000, 300, 6), (700, 1, 1)])
def test_select_matches_oracle(lib, m, n, F):
    rng = np.random.default_rng(m + n)
    s = gen.make_system(rng, m, n, noise=0.01, pad=np.nan)
    ref, marg = _margins(s, F)
    say("select", m, n, F, "min margin", min(marg) if marg else None)
    assert not marg or min(marg) > 1e-9
    g = lib.select(dev(s.Xt), dev(s.y), F)
    _check_selection(g, ref, F)
    check_a(g.a.cpu().numpy(), ref.a, tol=1e-6)


def test_select_planted_support_and_stop(lib):
    rng = np.random.default_rng(31)
    X = rng.standard_normal((4000, 90)).astype(np.float32)
    y = (5 * X[:, 3] - 4 * X[:, 71] + 3 * X[:, 40] + 0.01 * rng.standard_normal(4000)).astype(np.float32)
    Xt = np.ascontiguousarray(X.T)
    # (a noise column lowers ||e||^2 by about chi2_max / m ~ 0.25 %: under 1 %)
    g = lib.select(dev(Xt), dev(y), 10, tol=0.01)
    ref = oracle.select_features(Xt, y, 4000, F=10, tol=0.01)
    assert sorted(g.J) == [3, 40, 71] and g.J == ref.J and ref.stopped
    np.testing.assert_allclose(g.hist, ref.hist, rtol=1e-9)


def test_select_zero_columns_initial_guess_and_exhaustion(lib):
    rng = np.random.default_rng(8)
    s = gen.make_system(rng, 1500, 20, noise=0.01, pad=np.nan)
    s.Xt[[4, 11], :] = 0.0
    a0 = (0.5 * rng.standard_normal(s.n)).astype(np.float32)
    g = lib.select(dev(s.Xt), dev(s.y), 25, a0=dev(a0))
    ref = oracle.select_features(s.Xt, s.y, s.m, F=25, a0=a0.astype(np.float64))
    assert g.count == 18 and 4 not in g.J and 11 not in g.J
    _check_selection(g, ref, 25)
    check_a(g.a.cpu().numpy(), ref.a, tol=1e-6)


def test_select_wide_and_tall_full_size(lib):
    """Selection on the benchmark's tall (1M x 256) and wide (2000 x 200,000)
    systems: three choices each against the oracle."""
    for name, s in (("tall", gen.tall_large()), ("wide", gen.wide())):
        say("select full size", name)
        g = lib.select(dev(s.Xt), dev(s.y), 3)
        ref = oracle.select_features(s.Xt, s.y, s.m, F=3)
        _check_selection(g, ref, 3)


# ------------------------------------------------------------ benchmark configurations

def test_bench_config_rel_change_full_size(lib):
    """The 1M x 256 system exactly as the benchmark solves it (default kernel,
    relative change of ||e|| < 1e-6): the GPU stops within one sweep of the
    oracle's stop, and its coefficients, history and FP64 final check agree
    with the oracle run for the GPU's sweep count."""
    s = gen.tall_large()
    say("bench config: tall_large rel change")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=100, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    own = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, stop=oracle.STOP_REL_CHANGE, tol=1e-6)
    say("sweeps", r.info["sweeps_done"], own.sweeps, r.info)
    assert r.info["converged"] == 1 and abs(r.info["sweeps_done"] - own.sweeps) <= 1
    eq = own if own.sweeps == r.info["sweeps_done"] else oracle.solve(s.Xt, s.y, s.m,
                                                                      max_sweeps=r.info["sweeps_done"])
    check_a(r.a.cpu().numpy(), eq.a, info=r.info)
    check_hist(r.hist, eq.hist[: r.info["sweeps_done"] + 1])
    check_final(r, s, eq.a)


def test_bench_config_wide_fp32_equal_steps(lib):
    """Plain single precision on the full 2000 x 200,000 wide system, one
    sweep (200,000 column steps), against the oracle at equal steps."""
    s = gen.wide()
    say("bench config: wide fp32 one sweep")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=1)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=1)
    say("info", r.info, "ref hist", ref.hist)
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)
