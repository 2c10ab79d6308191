"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, after the same number of sweeps.

Bounds for single precision (the oracle runs on the FP32 input values):
* a: ||a_gpu - a_ora|| / ||a_ora|| <= 1e-5, and every coordinate
  |a_gpu,j - a_ora,j| <= 1e-5 ||a_ora||_inf;
* hist, sweep by sweep: |h_gpu[s] - h_ora[s]| <= 1e-5 h_ora[s] + 4 u h_ora[0]
  with u = 2^-24: the running residual is stored in FP32, so every entry
  carries a rounding error of the order of u times the entries it was
  formed from (|y_i| at the start); once ||e|| has fallen far below ||y||
  its norm is only resolved to about u ||y|| (the FP64 final check, below,
  is the exact value);
* final FP64 check: the reported ||y - X a|| / ||y|| equals the FP64 oracle's
  value for the returned coefficients to 1e-8 relative (1e-13 absolute: FP64
  sums in another order of terms up to ||y||), and differs from the
  oracle's own iterate's by at most ||X (a_gpu - a_ora)|| / ||y|| (triangle
  inequality).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

TOL_A = 1e-5
U32 = 2.0 ** -24


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def run(lib, s, sweeps, **kw):
    r = lib.solve(dev(s.Xt), dev(s.y), **({"a0": dev(kw.pop("a0"))} if "a0" in kw else {}), max_sweeps=sweeps, **kw)
    return r


def check_a(a, ref_a, tol=TOL_A, info=None):
    """Norm-wise and coordinate-wise agreement of the coefficients."""
    a = np.asarray(a, np.float64)
    ref_a = np.asarray(ref_a, np.float64)
    e = rel(a, ref_a)
    assert e <= tol, (e, info)
    scale = float(np.max(np.abs(ref_a))) if ref_a.size else 1.0
    worst = float(np.max(np.abs(a - ref_a))) / (scale if scale > 0 else 1.0) if a.size else 0.0
    assert worst <= tol, (worst, int(np.argmax(np.abs(a - ref_a))), info)


def check_hist(h, ref_hist):
    """Sweep-by-sweep agreement of ||e||, each entry against its own value."""
    h = np.asarray(h, np.float64)
    ref = np.asarray(ref_hist, np.float64)
    assert len(h) == len(ref), (len(h), len(ref))
    bound = 1e-5 * ref + 4 * U32 * ref[0]
    bad = np.flatnonzero(np.abs(h - ref) > bound)
    assert bad.size == 0, (bad[:5], h[bad[:5]], ref[bad[:5]])


def check_final(r, s, ref_a):
    """The FP64 final check: exact for the returned coefficients, and within
    the triangle-inequality bound of the oracle iterate's residual."""
    a = r.a.cpu().numpy().astype(np.float64)
    fr = r.info["final_rel_resid"]
    direct = oracle.final_rel_resid(s.Xt, s.y, s.m, a)
    # (FP64 sums in another order: 1e-8 relative, plus the rounding of terms
    # as large as ||y|| when the residual is far smaller)
    assert fr == pytest.approx(direct, rel=1e-8, abs=1e-13), (fr, direct)
    ynorm = np.linalg.norm(np.asarray(s.y[: s.m], np.float64))
    dx = np.linalg.norm(oracle.residual(s.Xt, np.zeros(s.m), s.m, a - ref_a))
    fr_ora = oracle.final_rel_resid(s.Xt, s.y, s.m, ref_a)
    assert abs(fr - fr_ora) <= dx / ynorm * (1 + 1e-6) + 1e-12 * fr_ora, (fr, fr_ora, dx / ynorm)


def check(lib, s, sweeps, tol=TOL_A, final=True, **kw):
    a0 = kw.get("a0")
    r = run(lib, s, sweeps, **kw)
    ref = oracle.solve(s.Xt, s.y, s.m, a0=a0, max_sweeps=sweeps)
    check_a(r.a.cpu().numpy(), ref.a, tol, r.info)
    assert len(r.hist) == sweeps + 1
    check_hist(r.hist, ref.hist)
    if final:
        check_final(r, s, ref.a)
    return r, ref


# ------------------------------------------------------------ exact cases

@pytest.mark.parametrize("flags", [0, 2])       # one workgroup / persistent grid
@pytest.mark.parametrize("block", [1, 2])
def test_dyadic_2x2_bitwise(lib, flags, block):
    """Closed form of Algorithm 1 on X = [[1,1],[0,1]], y = (2,1): all values
    dyadic, so the single-precision GPU result is exact."""
    say("dyadic", flags, block)
    Xt = np.zeros((2, 4), np.float32)
    Xt[0, :2] = [1, 0]
    Xt[1, :2] = [1, 1]
    Xt[:, 2:] = np.nan                             # padding rows are never read
    y = np.array([2, 1], np.float32)
    for s in (1, 2, 5, 12):
        r = lib.solve(dev(Xt), dev(y), max_sweeps=s, block=block, flags=flags)
        assert r.a.cpu().numpy().tolist() == [1 + 2.0 ** (1 - s), 1 - 2.0 ** (-s)]
        assert r.hist[-1] == math.sqrt(2.0) * 2.0 ** -s


# ------------------------------------------------------------ tall small

@pytest.mark.parametrize("team", ["wg", "grid"])
@pytest.mark.parametrize("block", [1, 4, 8])
def test_tall_small_200_sweeps(lib, team, block):
    s = gen.tall_small(pad=np.nan)
    flags = lib.F_FORCE_WG if team == "wg" else lib.F_FORCE_GRID
    say("tall_small", team, block)
    r, ref = check(lib, s, 200, block=block, flags=flags)
    assert r.info["block_used"] == block
    a_ls = np.linalg.lstsq(s.X(), s.y.astype(np.float64), rcond=None)[0]
    assert rel(r.a.cpu().numpy(), a_ls) < 1e-5
    assert r.info["final_rel_resid"] == pytest.approx(oracle.final_rel_resid(s.Xt, s.y, s.m, ref.a), rel=1e-4)


@pytest.mark.parametrize("m,n", [(1, 3), (5, 2), (7, 50), (1999, 37), (2001, 9), (4093, 21), (4096, 64),
                                 (4097, 13), (8193, 5)])
def test_ragged_shapes(lib, m, n):
    """Rows not a multiple of the 16-byte chunk, columns not a multiple of the
    block, NaN padding rows."""
    say("ragged", m, n)
    rng = np.random.default_rng(m * 1000 + n)
    s = gen.make_system(rng, m, n, noise=0.01, pad=np.nan)
    for flags in (0, lib.F_FORCE_GRID):
        check(lib, s, 15, flags=flags)


@pytest.mark.parametrize("m", [3, 4097, 8195])
@pytest.mark.parametrize("kind", [2, 3, 5, 8])
def test_grid_kinds_tiny_last_workgroup(lib, m, kind):
    """Grids whose last workgroup holds fewer valid rows than one chunk (or
    systems below one chunk), NaN padding rows: the chunks with no valid row
    must not bring the padding in."""
    say("tiny last workgroup", m, kind)
    rng = np.random.default_rng(m + kind)
    s = gen.make_system(rng, m, 21, noise=0.01, pad=np.nan)
    check(lib, s, 6, flags=lib.F_FORCE_GRID, depth=kind, block=16 if kind == 8 else (4 if kind < 5 else 8))


def test_tall_grid_multi_wg(lib):
    """Several hundred thousand rows: a persistent grid of many workgroups."""
    s = gen.tall_large(m=300_001, n=40, seed=7, pad=np.nan)
    say("tall grid 300001x40")
    for block in (1, 8):
        r, _ = check(lib, s, 4, block=block)
        assert r.info["team_wgs"] > 1


def test_tall_large_full_size_two_sweeps(lib):
    """The 1,000,000 x 256 bandwidth workload, in the launch configuration the
    benchmark uses, against the oracle after 2 sweeps."""
    s = gen.tall_large()
    say("tall_large full size")
    r, ref = check(lib, s, 2)
    say("info", r.info)
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] == 256
    for kind, tt, block in ((5, 256, 8), (5, 512, 4), (3, 512, 4)):
        say("grid kind", kind, tt, block)
        r, _ = check(lib, s, 2, depth=kind, team_threads=tt, block=block)
        assert r.info["kernel_kind"] == kind and r.info["team_threads"] == tt


def test_wide_workgroup(lib):
    s = gen.wide(m=2000, n=20000, seed=11)
    say("wide 2000x20000")
    r, ref = check(lib, s, 3)
    # consistent system: residual falls far below ||y||
    assert r.hist[-1] < 1e-2 * r.hist[0]


# ------------------------------------------------------------ semantics

def test_zero_columns_skipped(lib):
    rng = np.random.default_rng(3)
    s = gen.make_system(rng, 700, 12, noise=0.01)
    s.Xt[[2, 7], :] = 0.0
    say("zero columns")
    r, ref = check(lib, s, 30)
    assert r.info["zero_cols"] == 2 and ref.zero_cols == 2
    assert r.a.cpu().numpy()[2] == 0.0


@pytest.mark.parametrize("block,kind", [(16, 8), (8, 5)])
def test_grid_zero_and_correlated_columns(lib, block, kind):
    """Grid kernels on a system with zero columns and strongly correlated
    neighbours inside one column block: the block's steps (forward
    substitution, or its precomputed inverse for 16-column blocks) skip the
    zero columns and follow the sequential steps of Algorithm 1."""
    rng = np.random.default_rng(31)
    s = gen.make_system(rng, 100_003, 40, noise=0.01, pad=np.nan)
    s.Xt[[2, 7, 19], :] = 0.0
    s.Xt[5, :s.m] = 0.99 * s.Xt[4, :s.m] + 0.1 * s.Xt[6, :s.m]
    s.Xt[33, :s.m] = -s.Xt[32, :s.m] + 0.05 * s.Xt[34, :s.m]
    say("zero and correlated columns", kind)
    r, ref = check(lib, s, 8, flags=lib.F_FORCE_GRID, depth=kind, block=block)
    assert r.info["kernel_kind"] == kind and r.info["team_wgs"] > 1
    assert r.info["zero_cols"] == 3 and ref.zero_cols == 3
    assert np.all(r.a.cpu().numpy()[[2, 7, 19]] == 0.0)


def test_warm_start_resume(lib):
    """a0 = result of k sweeps, k more sweeps == 2k sweeps (to tolerance)."""
    s = gen.tall_small()
    say("warm start")
    r4 = run(lib, s, 4)
    r2 = run(lib, s, 2)
    rr = run(lib, s, 2, a0=r2.a.cpu().numpy())
    assert rel(rr.a.cpu().numpy(), r4.a.cpu().numpy()) < 1e-5
    check(lib, s, 3, a0=np.random.default_rng(1).standard_normal(s.n).astype(np.float32))


def test_hist_monotone(lib):
    s = gen.tall_large(m=200_000, n=64, seed=3)
    say("monotone")
    r = run(lib, s, 12)
    h = np.asarray(r.hist)
    assert np.all(h[1:] <= h[:-1] + 1e-6 * h[0])


def test_deterministic(lib):
    s = gen.tall_large(m=200_000, n=64, seed=3)
    say("deterministic")
    r1 = run(lib, s, 5)
    r2 = run(lib, s, 5)
    assert np.array_equal(r1.a.cpu().numpy(), r2.a.cpu().numpy())
    assert np.array_equal(r1.hist, r2.hist)


def test_stop_rel_change_matches_oracle(lib):
    s = gen.tall_small()
    say("stop rel change")
    r = run(lib, s, 200, stop=lib.STOP_REL_CHANGE, tol=1e-3)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=200, tol=1e-3, stop=oracle.STOP_REL_CHANGE)
    assert r.info["converged"] == 1 and r.info["sweeps_done"] == ref.sweeps
    assert rel(r.a.cpu().numpy(), ref.a) < TOL_A


def test_stop_rel_resid_with_column_checks(lib):
    s = gen.square_well_conditioned(64, seed=8)
    s32 = gen.System(s.Xt.astype(np.float32), s.y.astype(np.float32), 64, 64)
    say("stop rel resid")
    r = run(lib, s32, 500, stop=lib.STOP_REL_RESID, tol=1e-4, check_cols=8)
    ref = oracle.solve(s32.Xt, s32.y, 64, max_sweeps=500, tol=1e-4, stop=oracle.STOP_REL_RESID, check_cols=8)
    assert r.info["converged"] == 1
    assert r.info["cols_done"] == ref.cols
    assert rel(r.a.cpu().numpy(), ref.a) < TOL_A


def test_nonfinite_rejected(lib):
    s = gen.tall_small(m=300, n=10)
    s.Xt[3, 17] = np.inf
    say("nonfinite")
    with pytest.raises(lib.HPSCDError) as ei:
        run(lib, s, 3)
    assert ei.value.status == lib.ENONFINITE
    s = gen.tall_small(m=300, n=10)
    s.y[5] = np.nan
    with pytest.raises(lib.HPSCDError) as ei:
        run(lib, s, 3)
    assert ei.value.status == lib.ENONFINITE
    # the context stays usable
    check(lib, gen.tall_small(m=300, n=10), 3)


def test_zero_sweeps(lib):
    s = gen.tall_small(m=300, n=10)
    r = run(lib, s, 0)
    assert np.all(r.a.cpu().numpy() == 0) and len(r.hist) == 1
    assert r.hist[0] == pytest.approx(np.linalg.norm(s.y.astype(np.float64)), rel=1e-6)


def test_residual_f64(lib):
    s = gen.tall_small()
    a = np.random.default_rng(0).standard_normal(s.n).astype(np.float32)
    nrm, e = lib.residual_f64(dev(s.Xt), dev(s.y), dev(a), want_e=True)
    ref = oracle.residual(s.Xt, s.y, s.m, a.astype(np.float64))
    assert nrm == pytest.approx(np.linalg.norm(ref), rel=1e-12)
    np.testing.assert_allclose(e.cpu().numpy(), ref.astype(np.float32), rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------ pipelined grid

@pytest.mark.parametrize("block,kind", [(1, 2), (2, 2), (4, 2), (4, 3), (8, 3), (8, 5), (4, 5), (16, 8)])
def test_grid_kernel_kinds_match_oracle(lib, block, kind):
    """Every grid kernel kind (prefetch rings of two or three blocks; polling
    waves fed through LDS; 16-column blocks through the step matrix) produces
    the iterates of Algorithm 1 (n not a multiple of the block, ragged rows)."""
    s = gen.tall_large(m=300_003, n=37, seed=13, pad=np.nan)
    say("grid kind", block, kind)
    r, ref = check(lib, s, 6, block=block, depth=kind)
    assert r.info["block_used"] == block and r.info["team_wgs"] > 1


@pytest.mark.parametrize("m,team_threads", [(250_007, 256), (500_009, 512), (1_000_003, 512)])
def test_wide_kernel_default_shapes(lib, m, team_threads):
    """The default FP32 grid kernel (16-column blocks) takes the smallest
    workgroup shape that keeps the grid within 256 workgroups (capacity 1024
    rows up to ~262k rows, 2048 up to ~524k, then 4096) and spreads the rows
    evenly over up to one workgroup per CU.  Each shape follows Algorithm 1
    on a ragged system."""
    s = gen.tall_large(m=m, n=37, seed=17, pad=np.nan)
    say("wide default shape", m)
    r, ref = check(lib, s, 4)
    assert r.info["kernel_kind"] == 8 and r.info["team_threads"] == team_threads
    assert 245 <= r.info["team_wgs"] <= 256  # (rows spread over up to one workgroup per CU)


@pytest.mark.parametrize("m,n", [(2000, 200), (1500, 37), (700, 64), (4000, 48), (5, 20)])
def test_wide_kernel_one_workgroup(lib, m, n):
    """The wide-block kernel as a single workgroup (no grid exchange: the
    workgroup's sums are the totals), 16-column blocks through the step
    matrix, n not always a multiple of 16, NaN padding rows."""
    rng = np.random.default_rng(m + n)
    s = gen.make_system(rng, m, n, noise=0.01, pad=np.nan)
    say("wide one workgroup", m, n)
    r, ref = check(lib, s, 12, block=16, depth=8)
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] == 1


def test_wide_kernel_one_workgroup_resid_stop(lib):
    """The single-workgroup wide kernel stops at a column check inside a
    sweep where the oracle does."""
    s = gen.tall_small(n=48, pad=np.nan)
    say("wide one workgroup resid stop")
    kw = dict(stop=lib.STOP_REL_RESID, tol=0.01, check_cols=16)
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=50, block=16, depth=8, **kw)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=50, stop=oracle.STOP_REL_RESID, tol=0.01, check_cols=16)
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] == 1
    assert r.info["converged"] == 1 and r.info["cols_done"] == ref.cols
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5


def test_ring_grid_stop_rule(lib):
    s = gen.tall_large(m=250_000, n=48, seed=21)
    say("ring grid stop")
    r = run(lib, s, 100, block=4, depth=3, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, tol=1e-6, stop=oracle.STOP_REL_CHANGE)
    assert r.info["converged"] == 1 and abs(r.info["sweeps_done"] - ref.sweeps) <= 1
    check(lib, s, r.info["sweeps_done"], block=4, depth=3)


def test_ring_grid_warm_start(lib):
    s = gen.tall_large(m=200_000, n=24, seed=5)
    a0 = np.random.default_rng(2).standard_normal(s.n).astype(np.float32)
    say("ring grid warm")
    check(lib, s, 3, a0=a0, block=4, depth=3)


def test_depth4_is_one_workgroup_only(lib):
    s = gen.tall_small(m=300, n=10)
    with pytest.raises(lib.HPSCDError) as ei:
        run(lib, s, 2, block=4, depth=4, flags=lib.F_FORCE_GRID)
    assert ei.value.status == lib.EINVAL


@pytest.mark.parametrize("team_threads", [256, 512])
def test_polling_wave_kernel_shapes(lib, team_threads):
    """The polling-wave kernel with one (512 x 2, block 4) or two (256 x 4,
    block 8) polling waves, whose rows reach them through LDS, against the
    oracle on a ragged system with a warm start and the relative-change stop."""
    s = gen.tall_large(m=200_001, n=45, seed=21, pad=np.nan)
    block = 8 if team_threads == 256 else 4
    say("px", team_threads, block)
    rng = np.random.default_rng(3)
    a0 = rng.standard_normal(s.n).astype(np.float32)
    r = lib.solve(dev(s.Xt), dev(s.y), dev(a0), max_sweeps=30, stop=lib.STOP_REL_CHANGE, tol=1e-5, block=block,
                  depth=5, team_threads=team_threads, flags=lib.F_FORCE_GRID)
    ref = oracle.solve(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=30, stop=oracle.STOP_REL_CHANGE, tol=1e-5)
    assert abs(r.info["sweeps_done"] - ref.sweeps) <= 1
    ref_eq = oracle.solve(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=r.info["sweeps_done"])
    assert rel(r.a.cpu().numpy(), ref_eq.a) <= 1e-5
    assert r.info["team_threads"] == team_threads and r.info["team_wgs"] > 1


@pytest.mark.parametrize("kind,team_threads,m,n,stop", [(5, 512, 200_001, 45, "change"), (5, 512, 100_003, 48, "resid"),
                                                         (8, 512, 200_001, 45, "change"), (8, 512, 100_003, 48, "resid")])
def test_blocks_in_flight_kernel(lib, kind, team_threads, m, n, stop):
    """The polling-wave grid kernel (kind 5, 8-column blocks) and the
    wide-block kernel (kind 8, 16 columns per reduction), on ragged systems
    with a warm start, stopping inside the loop:
    on the relative change of ||e|| at a sweep end, or on the relative
    residual at a column check inside a sweep.  The stop lands where the
    oracle's does and the iterate matches the oracle's after as many steps."""
    s = gen.tall_large(m=m, n=n, seed=29, pad=np.nan)
    say("pe", kind, team_threads, m, stop)
    rng = np.random.default_rng(4)
    a0 = rng.standard_normal(s.n).astype(np.float32)
    if stop == "change":
        kw, okw = dict(stop=lib.STOP_REL_CHANGE, tol=1e-5), dict(stop=oracle.STOP_REL_CHANGE, tol=1e-5)
    else:
        cc = 16 if kind == 8 else 8  # (the block divides check_cols)
        kw = dict(stop=lib.STOP_REL_RESID, tol=0.015, check_cols=cc)
        okw = dict(stop=oracle.STOP_REL_RESID, tol=0.015, check_cols=cc)
    r = lib.solve(dev(s.Xt), dev(s.y), dev(a0), max_sweeps=30, block=16 if kind == 8 else 8, depth=kind,
                  team_threads=team_threads, flags=lib.F_FORCE_GRID, **kw)
    ref = oracle.solve(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=30, **okw)
    assert r.info["kernel_kind"] == kind and r.info["team_wgs"] > 1
    assert r.info["converged"] == 1
    if stop == "change":
        assert abs(r.info["sweeps_done"] - ref.sweeps) <= 1
        ref_eq = oracle.solve(s.Xt, s.y, s.m, a0=a0.astype(np.float64), max_sweeps=r.info["sweeps_done"])
        assert rel(r.a.cpu().numpy(), ref_eq.a) <= 1e-5
    else:
        assert r.info["cols_done"] == ref.cols and ref.cols % n != 0  # a check inside a sweep
        assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5


@pytest.mark.parametrize("m,n,kw", [(1_000_000, 256, {}), (2000, 512, dict(block=16, depth=8)),
                                    (2000, 4096, dict(depth=9))])
def test_abort_from_another_thread(lib, m, n, kw):
    """hpscd_abort from a second host thread ends a running solve at the next
    sweep start with EABORTED (the grid kernel, the wide-block kernel as one
    workgroup, the column chain); the solve is bounded (4000 sweeps), so a
    missed request shows as a failure, not a hang."""
    import threading
    import time
    import torch
    rng = np.random.default_rng(m + n)
    s = gen.make_system(rng, m, n, noise=0.01)
    X, y = dev(s.Xt), dev(s.y)
    torch.cuda.synchronize()
    say("abort", m, n)
    box = {}

    def run():
        try:
            box["r"] = lib.solve(X, y, max_sweeps=4000, **kw)
        except lib.HPSCDError as ex:
            box["e"] = ex

    t = threading.Thread(target=run)
    t.start()
    time.sleep(0.15)
    lib.abort()
    t.join(120)
    assert not t.is_alive()
    assert "e" in box and box["e"].status == lib.EABORTED, box


@pytest.mark.parametrize("n,warm", [(1, False), (2, False), (17, False), (33, True)])
def test_wide_grid_few_columns(lib, n, warm):
    """The wide-block grid with fewer columns than one block, one column past
    a block, and a warm start: the next block's first two columns, requested
    after each exchange, are the block's own again when a sweep has one
    block (n <= 16), and the last valid column when the block holds one."""
    rng = np.random.default_rng(100 + n)
    s = gen.make_system(rng, 200_000, n, noise=0.01, pad=np.nan)
    a0 = rng.standard_normal(n).astype(np.float32) if warm else None
    say("wide grid few columns", n, warm)
    r, _ = check(lib, s, 6, depth=8, flags=lib.F_FORCE_GRID, **({"a0": a0} if warm else {}))
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] > 1


@pytest.mark.parametrize("kw", [dict(depth=8), dict(depth=5, block=8), dict(depth=2, block=8),
                                dict(depth=3, block=8)])
def test_spin_timeout_ends_the_solve(lib, kw):
    """A bound of 1 us on the grid waits (the first poll then follows the
    publish after 0.5 us, before the slowest workgroups have published) ends
    the solve with ETIMEOUT, on every grid kernel: every workgroup's wait is
    bounded, so the kernel exits normally; the next solve on the context runs
    as if nothing happened."""
    s = gen.tall_large()
    X, y = dev(s.Xt), dev(s.y)
    say("spin timeout", kw)
    ref = lib.solve(X, y, max_sweeps=3, **kw)
    assert ref.info["team_wgs"] > 1 and ref.info["kernel_kind"] == kw["depth"]
    with pytest.raises(lib.HPSCDError) as ei:
        lib.solve(X, y, max_sweeps=3, spin_timeout_us=1, **kw)
    assert ei.value.status == lib.ETIMEOUT
    again = lib.solve(X, y, max_sweeps=3, **kw)
    assert np.array_equal(again.a.cpu().numpy(), ref.a.cpu().numpy())
    assert np.array_equal(again.hist, ref.hist)


def test_abort_before_solve_is_dropped(lib):
    """A cancel request made while no solve runs does not end the next one."""
    s = gen.tall_small(m=3000, n=40)
    lib.abort()
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3)
    assert r.info["sweeps_done"] == 3


# ------------------------------------------------ memory past the last column

def _nan_tailed(Xt):
    """Xt (n, ldx) on the GPU as the first n rows of an (n + 16, ldx) tensor
    whose 16 rows after it (the memory past column n - 1) are NaN: a kernel
    that reads a column past n would turn the result non-finite."""
    import torch
    n, ldx = Xt.shape
    big = torch.full((n + 16, ldx), float("nan"), dtype=torch.float32, device="cuda")
    big[:n] = torch.from_numpy(np.ascontiguousarray(Xt)).cuda()
    return big[:n]


@pytest.mark.parametrize("kind,m,kw", [
    (9, 1500, dict(depth=9)),
    (8, 3000, dict(depth=8, block=16, flags=4)),
    (8, 100_003, dict(depth=8, block=16)),
    (5, 200_001, dict(depth=5, block=8, flags=2)),
    (2, 50_001, dict(depth=2, block=8, flags=2)),
    (3, 50_001, dict(depth=3, block=4, flags=2)),
    (2, 3000, dict(depth=2, block=4, flags=4)),
])
def test_no_read_past_last_column(lib, kind, m, kw):
    """n = 37 (not a multiple of 4, 8 or 16): the last block's missing columns
    re-read its last valid column, never the NaN memory that follows X."""
    rng = np.random.default_rng(kind * 7 + m)
    s = gen.make_system(rng, m, 37, noise=0.01, pad=np.nan)
    say("past last column", kind, m)
    r = lib.solve(_nan_tailed(s.Xt), dev(s.y), max_sweeps=3, **kw)
    assert r.info["kernel_kind"] == kind
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=3)
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)
    check_hist(r.hist, ref.hist)
    check_final(r, s, ref.a)


def test_bf16_chain_no_read_past_last_column(lib):
    s = gen.make_system(np.random.default_rng(5), 2000, 45, noise=0.01, pad=np.nan)
    import torch
    X32 = dev(s.Xt)
    xb = lib.convert_bf16(X32)
    n, ldd = xb.shape
    bigb = torch.full((n + 16, ldd), float("nan"), dtype=torch.bfloat16, device="cuda")
    bigb[:n] = xb
    r = lib.solve_bf16(bigb[:n], X32, dev(s.y), max_sweeps=4, depth=9)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=4)
    assert r.info["kernel_kind"] == 9 and r.info["block_used"] == 32
    check_a(r.a.cpu().numpy(), ref.a, info=r.info)


def test_batched_no_read_past_last_column(lib):
    """The batched kernel on a pool followed by NaN memory, every system with
    n not a multiple of the block."""
    import torch
    b = gen.batch(seed=31, count=24, m_lo=256, m_hi=8192, n_lo=5, n_hi=61, pad=np.nan)
    pool = torch.full((b.Xpool.size + 4096,), float("nan"), dtype=torch.float32, device="cuda")
    pool[: b.Xpool.size] = torch.from_numpy(b.Xpool).cuda()
    say("batched past last column", b.count)
    for block in (1, 2, 4):
        r = lib.solve_batched(pool[: b.Xpool.size], dev(b.ypool), b.table, max_sweeps=6, block=block)
        a = r.a.cpu().numpy()
        for i in range(b.count):
            sys_ = b.system(i)
            ao = b.table[i, 5]
            ref = oracle.solve(sys_.Xt, sys_.y, sys_.m, max_sweeps=6)
            check_a(a[ao: ao + sys_.n], ref.a, info=(block, i))
