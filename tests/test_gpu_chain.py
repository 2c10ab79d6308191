"""GPU parity of the column-chain kernel (kernel kind 9): Algorithm 1 on a
short system (at most 2048 rows) as one workgroup, 16 FP32 or 32 bfloat16
columns per block through each block's step matrix, against the FP64
oracle (the same bounds as test_gpu_parity; the storage form against the
oracle of that form).  Sizes span several blocks, a ragged last block
(n not a multiple of the block), ragged rows (m not a multiple of 4, rows
past m NaN-padded) and the edge cases m = 1, n = 1 and zero sweeps.
"""
import numpy as np
import pytest

import oracle
from workloads import gen

from test_gpu_parity import check, check_a, check_final, check_hist, dev, rel, say

pytestmark = pytest.mark.gpu


def bf16_pair(lib, s):
    X32 = dev(s.Xt)
    return lib.convert_bf16(X32), X32


# ------------------------------------------------------------------ FP32

@pytest.mark.parametrize("m,n", [(2000, 200), (1500, 37), (2048, 100), (700, 64), (5, 20), (1, 3), (333, 1),
                                 (2047, 16)])
def test_chain_f32_matches_oracle(lib, m, n):
    rng = np.random.default_rng(7 * m + n)
    s = gen.make_system(rng, m, n, noise=0.01, pad=np.nan)
    say("chain f32", m, n)
    r, _ = check(lib, s, 12, depth=9)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 16 and r.info["team_wgs"] == 1


def test_chain_is_default_for_short_systems(lib):
    s = gen.tall_small(pad=np.nan)
    say("chain default")
    r, _ = check(lib, s, 20)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 16
    # options the chain cannot take fall back to the other kernels
    r, _ = check(lib, s, 5, block=8)
    assert r.info["kernel_kind"] != 9 and r.info["block_used"] == 8
    s2 = gen.tall_small(m=2049, n=40, pad=np.nan)
    r, _ = check(lib, s2, 5)
    assert r.info["kernel_kind"] != 9


def test_chain_warm_start(lib):
    s = gen.tall_small(n=70, pad=np.nan)
    a0 = np.random.default_rng(3).standard_normal(s.n).astype(np.float32)
    say("chain a0")
    check(lib, s, 4, depth=9, a0=a0)


def test_chain_zero_sweeps(lib):
    s = gen.tall_small(m=300, n=10)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=0, depth=9)
    assert np.all(r.a.cpu().numpy() == 0) and len(r.hist) == 1
    assert r.hist[0] == pytest.approx(np.linalg.norm(s.y.astype(np.float64)), rel=1e-6)


def test_chain_stop_rel_change(lib):
    s = gen.tall_small()
    say("chain rel change")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=200, stop=lib.STOP_REL_CHANGE, tol=1e-3, depth=9)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200, tol=1e-3, stop=oracle.STOP_REL_CHANGE)
    assert r.info["converged"] == 1 and r.info["sweeps_done"] == ref.sweeps
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)


def test_chain_stop_rel_resid_inside_sweep(lib):
    """A column check inside a sweep (every 32 columns of 96) stops where the
    oracle's does."""
    s = gen.square_well_conditioned(96, seed=8)
    s32 = gen.System(s.Xt.astype(np.float32), s.y.astype(np.float32), 96, 96)
    say("chain rel resid")
    kw = dict(stop=lib.STOP_REL_RESID, tol=1e-4, check_cols=32)
    r = lib.solve(dev(s32.Xt), dev(s32.y), max_sweeps=500, depth=9, **kw)
    ref = oracle.solve(s32.Xt, s32.y, 96, max_sweeps=500, tol=1e-4, stop=oracle.STOP_REL_RESID, check_cols=32)
    assert r.info["kernel_kind"] == 9
    assert r.info["converged"] == 1 and ref.converged
    assert r.info["cols_done"] == ref.cols
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)


def test_chain_rel_grad_stop(lib):
    s = gen.tall_small(pad=np.nan)
    say("chain rel grad")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=100, stop=lib.STOP_REL_GRAD, tol=1e-4, depth=9)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, stop=oracle.STOP_REL_GRAD, tol=1e-4)
    assert r.info["kernel_kind"] == 9
    assert r.info["converged"] == 1 and r.info["sweeps_done"] == ref.sweeps
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)


def test_chain_nonfinite(lib):
    s = gen.tall_small(m=300, n=40)
    s.Xt[33, 17] = np.nan
    with pytest.raises(lib.HPSCDError) as ei:
        lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, depth=9)
    assert ei.value.status == lib.ENONFINITE
    check(lib, gen.tall_small(m=300, n=40), 3, depth=9)


def test_chain_rejections(lib):
    s = gen.tall_small(m=2100, n=40)
    for kw in (dict(depth=9), dict(depth=9, block=16, flags=lib.F_FORCE_GRID),
               dict(block=32), dict(depth=9, team_threads=256)):
        with pytest.raises(lib.HPSCDError) as ei:
            lib.solve(dev(s.Xt), dev(s.y), max_sweeps=2, **kw)
        assert ei.value.status == lib.EINVAL, kw
    s = gen.tall_small(m=500, n=40)
    for kw in (dict(block=32), dict(depth=9, stop=lib.STOP_REL_RESID, tol=1e-3, check_cols=24),
               dict(depth=9, thr=4)):
        with pytest.raises(lib.HPSCDError) as ei:
            lib.solve(dev(s.Xt), dev(s.y), max_sweeps=2, **kw)
        assert ei.value.status == lib.EINVAL, kw


def test_chain_deterministic(lib):
    s = gen.wide(m=2000, n=4000, seed=11)
    r1 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, depth=9)
    r2 = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, depth=9)
    assert np.array_equal(r1.a.cpu().numpy(), r2.a.cpu().numpy())
    assert np.array_equal(r1.hist, r2.hist)


# ------------------------------------------------------------- bfloat16

@pytest.mark.parametrize("m,n,refresh", [(2000, 480, 160), (1500, 37, 0), (2000, 8000, 4000), (7, 70, 0),
                                         (2048, 64, 32)])
def test_chain_bf16_matches_oracle(lib, m, n, refresh):
    rng = np.random.default_rng(m + 3 * n)
    s = gen.make_system(rng, m, n, noise=0.01, pad=np.nan)
    Xb, X32 = bf16_pair(lib, s)
    sweeps = 3 if n > 1000 else 8
    say("chain bf16", m, n, refresh)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=sweeps, refresh_cols=refresh, depth=9)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=sweeps, refresh_cols=refresh)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 32
    assert r.info["refreshes"] == ref.refreshes
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)


def test_chain_bf16_is_default(lib):
    s = gen.wide(m=2000, n=3200, seed=12)
    Xb, X32 = bf16_pair(lib, s)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=2, refresh_cols=1600)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=2, refresh_cols=1600)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 32
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)


@pytest.mark.parametrize("size", ["mid", "full"])
def test_chain_bf16_time_to_tolerance(lib, size):
    """The relative-residual stop of the storage form on the wide system, in
    the configuration the benchmark times for "full" (2000 x 200,000; check
    every 1024 columns, refresh every 16384, tol 1e-6): the stop is
    confirmed on the refreshed residual, lands on the oracle's column check
    after the oracle's refreshes, and the iterates agree there."""
    if size == "mid":
        s = gen.wide(m=2000, n=20_000, seed=5)
        tol, check_cols, refresh = 1e-6, 512, 2048
    else:
        s = gen.wide()
        tol, check_cols, refresh = 1e-6, 1024, 16384
    Xb, X32 = bf16_pair(lib, s)
    say("chain bf16 confirm", size)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=3, stop=lib.STOP_REL_RESID, tol=tol, check_cols=check_cols,
                       refresh_cols=refresh)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=3, stop=oracle.STOP_REL_RESID, tol=tol,
                                    check_cols=check_cols, refresh_cols=refresh)
    say("cols", r.info["cols_done"], ref.cols, "refreshes", r.info["refreshes"], ref.refreshes)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 32
    assert ref.converged and r.info["converged"] == 1
    assert r.info["final_rel_resid"] < tol
    assert r.info["cols_done"] == ref.cols
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5


def test_chain_f32_full_size_wide(lib):
    """The FP32 form on the 2000 x 200,000 system as the benchmark runs it
    (relative-residual stop 1e-6 checked every 1024 columns): stop point and
    iterate against the oracle."""
    s = gen.wide()
    say("chain f32 full")
    kw = dict(stop=lib.STOP_REL_RESID, tol=1e-6, check_cols=1024)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, **kw)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=3, stop=oracle.STOP_REL_RESID, tol=1e-6, check_cols=1024)
    assert r.info["kernel_kind"] == 9
    assert r.info["converged"] == 1 and ref.converged
    assert r.info["cols_done"] == ref.cols
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
