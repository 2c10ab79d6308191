"""GPU parity of the bfloat16-storage form and of the batched form."""
import numpy as np
import pytest

import oracle
from oracle import hpscd_oracle as ho
from workloads import gen

pytestmark = pytest.mark.gpu


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


# ---------------------------------------------------------------- bfloat16

def test_convert_bf16_bitwise(lib):
    """GPU rounding to bfloat16 equals the oracle's (and torch's) on every value."""
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000), rng.standard_normal(500) * 1e-39,
                        rng.standard_normal(500) * 1e37, [0.0, -0.0, np.inf, -np.inf]]).astype(np.float32)
    u = x.view(np.uint32)
    ties = ((u & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties[:1000]])
    n = 7
    m = len(x) // n
    Xt = np.zeros((n, gen.round_up(m, 8)), np.float32)
    Xt[:, :m] = x[: n * m].reshape(n, m)
    got = lib.convert_bf16(dev(Xt)).view(torch.int16).cpu().numpy().view(np.uint16)
    ref = (ho.bf16_round(Xt).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(got[:, :m], ref[:, :m])


@pytest.mark.parametrize("team", ["wg", "grid"])
def test_bf16_form_matches_oracle(lib, team):
    """The storage form against the oracle of the same form (Algorithm 1 on
    bfloat16-rounded X, residual refreshed from FP32 X every refresh_cols
    column steps) at equal sweeps."""
    if team == "wg":
        s = gen.wide(m=2000, n=8000, seed=5)
        flags, refresh, sweeps = lib.F_FORCE_WG, 4000, 3
    else:
        s = gen.tall_large(m=100_000, n=32, seed=9)
        flags, refresh, sweeps = lib.F_FORCE_GRID, 32, 4
    say("bf16", team)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=sweeps, refresh_cols=refresh, flags=flags)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=sweeps, refresh_cols=refresh)
    assert r.info["refreshes"] >= 1
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5, r.info
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])
    fr = oracle.final_rel_resid(s.Xt, s.y, s.m, ref.a)
    assert r.info["final_rel_resid"] == pytest.approx(fr, rel=1e-3, abs=1e-7)


def test_bf16_no_refresh_error_bound(lib):
    """Without refresh the error against the FP32 problem is that of the
    rounded matrix: stated per result, here bounded by 2^-7 relative in a."""
    s = gen.tall_small()
    X32 = dev(s.Xt)
    r = lib.solve_bf16(lib.convert_bf16(X32), X32, dev(s.y), max_sweeps=100)
    ref32 = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100)
    refb = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=100)
    assert rel(r.a.cpu().numpy(), refb.a) <= 1e-5
    assert rel(r.a.cpu().numpy(), ref32.a) <= 2.0 ** -7


# ---------------------------------------------------------------- batched

@pytest.mark.parametrize("block", [1, 2, 4])
def test_batched_matches_oracle(lib, block):
    b = gen.batch(seed=4, count=40, m_lo=100, m_hi=8192, n_lo=3, n_hi=128, pad=np.nan)
    say("batched", block, b.count)
    r = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, max_sweeps=12, block=block, want_hist=True)
    a = r.a.cpu().numpy()
    refs = oracle.solve_batch(b, max_sweeps=12)
    for i, ref in enumerate(refs):
        m, n, _, _, _, ao = b.table[i]
        assert rel(a[ao: ao + n], ref.a) <= 1e-5, (i, m, n)
        assert r.sweeps[i] == 12
        assert np.all(np.abs(r.hist[i] - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])
        fr = oracle.final_rel_resid(b.system(i).Xt, b.system(i).y, m, ref.a)
        assert r.final_rel_resid[i] == pytest.approx(fr, rel=1e-3, abs=1e-7)


def test_batched_equals_single(lib):
    b = gen.batch(seed=6, count=16, m_lo=256, m_hi=8192, n_lo=8, n_hi=64)
    r = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, max_sweeps=8)
    a = r.a.cpu().numpy()
    for i in range(b.count):
        s = b.system(i)
        one = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=8).a.cpu().numpy()
        ao = b.table[i, 5]
        assert rel(a[ao: ao + s.n], one) <= 1e-5


def test_batched_tuned_order_changes_no_result(lib):
    """The autotuner's cost order (sweeps recorded on the live batch) hands
    out the systems in another order than an untuned call; every system is
    solved by one team either way, so a, sweeps and the FP64 check are the
    same bit for bit (same kernel variant: block 4, eight-wave workgroups;
    every system above one wave's rows, so each is a workgroup team under
    any work split)."""
    b = gen.batch(seed=12, count=300, m_lo=1100, m_hi=8192, n_lo=8, n_hi=128)
    Xp, yp = dev(b.Xpool), dev(b.ypool)
    kw = dict(max_sweeps=60, stop=lib.STOP_REL_CHANGE, tol=1e-6, block=4, team_threads=512)
    before = lib.solve_batched(Xp, yp, b.table, **kw)
    lib.autotune_batched(Xp, yp, b.table, max_sweeps=60, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    after = lib.solve_batched(Xp, yp, b.table, **kw)
    assert np.array_equal(before.a.cpu().numpy(), after.a.cpu().numpy())
    assert np.array_equal(before.sweeps, after.sweeps)
    assert np.array_equal(before.final_rel_resid, after.final_rel_resid)


def test_batched_stop_and_warm_start(lib):
    b = gen.batch(seed=8, count=24, m_lo=256, m_hi=4096, n_lo=8, n_hi=64)
    say("batched stop")
    r = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, max_sweeps=200,
                          stop=lib.STOP_REL_CHANGE, tol=1e-6)
    refs = oracle.solve_batch(b, max_sweeps=200, tol=1e-6, stop=oracle.STOP_REL_CHANGE)
    agree = sum(int(r.sweeps[i] == refs[i].sweeps) for i in range(b.count))
    assert agree >= b.count - 2          # a sweep count may differ right at the threshold
    assert np.all(r.converged == 1)
    # warm start from the converged answer: the residual does not grow
    a0 = r.a.clone()
    r2 = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, a0pool=a0, max_sweeps=1, want_hist=True)
    for i in range(b.count):
        assert r2.hist[i][1] <= r2.hist[i][0] * (1 + 1e-6)


def test_bf16_ring_refresh_mid_sweep(lib):
    """Refresh every 16 column steps on a 32-column system: each launch of the
    grid kernel ends inside a sweep, and the next one starts from the
    refreshed residual."""
    s = gen.tall_large(m=100_000, n=32, seed=9)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    say("bf16 ring mid sweep")
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=4, refresh_cols=16, block=4, depth=2)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=4, refresh_cols=16)
    assert r.info["refreshes"] == ref.refreshes == 8
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5, r.info
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])


@pytest.mark.parametrize("size", ["mid", "full"])
def test_bf16_time_to_tolerance_is_confirmed(lib, size):
    """Relative-residual stop of the storage form on the wide system: the
    stop is confirmed on the residual recomputed from FP32 X, so the FP64
    final check is under tol; stop point and refresh count follow the oracle.
    "full" is the 2000 x 200,000 system in the configuration the benchmark
    times (check every 1024 columns, refresh every 16384)."""
    if size == "mid":
        s = gen.wide(m=2000, n=20_000, seed=5)
        tol, check, refresh = 1e-6, 512, 2048
    else:
        s = gen.wide()
        tol, check, refresh = 1e-6, 1024, 16384
    say("bf16 confirm", size)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=3, stop=lib.STOP_REL_RESID, tol=tol, check_cols=check,
                       refresh_cols=refresh, block=8)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=3, stop=oracle.STOP_REL_RESID, tol=tol,
                                    check_cols=check, refresh_cols=refresh)
    say("cols", r.info["cols_done"], ref.cols, "refreshes", r.info["refreshes"], ref.refreshes)
    assert ref.converged and r.info["converged"] == 1
    assert r.info["final_rel_resid"] < tol
    # the stop lands on the same column check, after the same refreshes, and
    # the iterates agree there
    assert r.info["cols_done"] == ref.cols
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5


def test_batched_graph_replays_match_eager(lib):
    """The recorded batched solve, replayed several times with eager work and
    host waits in between, gives the eager call's results every time; a new
    a0 written into the bound pool is picked up by the next replay."""
    import torch
    b = gen.batch(seed=14, count=48, m_lo=200, m_hi=8192, n_lo=4, n_hi=100)
    Xp, yp = dev(b.Xpool), dev(b.ypool)
    say("graph plan")
    eager = lib.solve_batched(Xp, yp, b.table, max_sweeps=15, stop=lib.STOP_REL_CHANGE, tol=1e-6, want_hist=True)
    a0 = torch.zeros(eager.a.numel(), dtype=torch.float32, device="cuda")
    plan = lib.BatchPlan(Xp, yp, b.table, a0pool=a0, max_sweeps=15, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    for rep in range(3):
        plan.launch()
        got = plan.results(want_hist=True)
        assert torch.equal(got.a, eager.a), rep
        assert np.array_equal(got.sweeps, eager.sweeps)
        assert np.array_equal(got.hist, eager.hist, equal_nan=True)
        np.testing.assert_allclose(got.final_rel_resid, eager.final_rel_resid, rtol=1e-12)
        # unrelated eager work between replays
        lib.solve_batched(Xp, yp, b.table, max_sweeps=2)
        torch.cuda.synchronize()
    a0.copy_(eager.a)  # warm start from the converged answer through the bound pool
    warm = lib.solve_batched(Xp, yp, b.table, a0pool=a0.clone(), max_sweeps=15, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    plan.launch()
    got = plan.results()
    assert torch.equal(got.a, warm.a)
    assert np.array_equal(got.sweeps, warm.sweeps)
    plan.close()


def test_batched_full_size_sampled(lib):
    """The 4096-system batch in the configuration the benchmark times
    (autotuned, recorded as a graph, relative-change stop 1e-6): sampled
    systems (the largest, the smallest, and random ones) against the oracle
    run for the sweep count the GPU reports, and against the oracle's own stop."""
    b = gen.batch()
    Xp, yp = dev(b.Xpool), dev(b.ypool)
    kw = dict(max_sweeps=100, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    say("batched full size: autotune")
    lib.autotune_batched(Xp, yp, b.table, **kw)
    plan = lib.BatchPlan(Xp, yp, b.table, **kw)
    plan.launch()
    r = plan.results()
    a = r.a.cpu().numpy()
    assert np.all(r.converged == 1)
    work = b.table[:, 0] * b.table[:, 1]
    order = np.argsort(work)
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([order[:6], order[-6:], rng.choice(b.count, 12, replace=False)]))
    for i in sample:
        s = b.system(int(i))
        ao = b.table[i, 5]
        ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=int(r.sweeps[i]))
        assert rel(a[ao: ao + s.n], ref.a) <= 1e-5, (i, s.m, s.n)
        own = oracle.solve(s.Xt, s.y, s.m, max_sweeps=100, stop=oracle.STOP_REL_CHANGE, tol=1e-6)
        assert abs(own.sweeps - int(r.sweeps[i])) <= 1, (i, own.sweeps, r.sweeps[i])


@pytest.mark.parametrize("team_threads,block", [(256, 0), (512, 1), (512, 2), (512, 4)])
def test_batched_size_boundaries(lib, team_threads, block):
    """Systems at the edges of the batched kernel's work split in both
    workgroup shapes: m = 1024 and 2048 (the largest that one wave holds with
    four and eight chunks per thread), 1025 and 2049, 8192 (the largest
    accepted), tiny m, n = 1 and n close to m; more small systems than a
    workgroup has waves, so items of wave teams are full and one is partial."""
    rng = np.random.default_rng(77)
    sizes = [(1024, 40), (1025, 40), (2048, 40), (2049, 40), (8192, 100), (8192, 1), (2, 1), (3, 2), (100, 90),
             (64, 50), (1000, 7), (500, 30), (300, 12), (700, 64), (900, 5), (256, 255)]
    systems = [gen.make_system(rng, m, n, noise=0.01, pad=np.nan) for m, n in sizes]
    b = gen.pack(systems)
    say("batched boundaries", team_threads, block)
    r = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, max_sweeps=20, want_hist=True,
                          team_threads=team_threads, block=block)
    assert r.info["team_threads"] == team_threads
    a = r.a.cpu().numpy()
    for i, s in enumerate(systems):
        ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=20)
        ao = b.table[i, 5]
        assert rel(a[ao: ao + s.n], ref.a) <= 1e-5, sizes[i]
        assert np.all(np.abs(r.hist[i] - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0]), sizes[i]


def test_bf16_polling_wave_kernel(lib):
    """The storage form through the polling-wave grid kernel (kind 5), with
    refreshes between launch segments, against the oracle of the form."""
    s = gen.tall_large(m=150_000, n=40, seed=23)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    say("bf16 px")
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=4, refresh_cols=40, block=8, depth=5, team_threads=512,
                       flags=lib.F_FORCE_GRID)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=4, refresh_cols=40)
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])


@pytest.mark.parametrize("kind", [3, 8])
def test_bf16_grid_kernel_kinds(lib, kind):
    """The storage form through the grid kernel with a ring of three column
    blocks (kind 3) and through the wide-block kernel (kind 8), with
    refreshes between launch segments, against the oracle of the form."""
    s = gen.tall_large(m=150_000, n=48 if kind == 8 else 40, seed=23)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    say("bf16 pe", kind)
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=4, refresh_cols=80 if kind == 8 else 40,
                       block=16 if kind == 8 else 8, depth=kind, team_threads=512, flags=lib.F_FORCE_GRID)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=4, refresh_cols=80 if kind == 8 else 40)
    assert r.info["kernel_kind"] == kind
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])


def test_bf16_wide_kernel_spread_grid(lib):
    """The storage form on the wide-block kernel with its rows spread over
    one workgroup per CU (about 3,900 rows each, ragged last workgroup, NaN
    padding rows), with refreshes, against the oracle of the form."""
    s = gen.tall_large(m=1_000_003, n=32, seed=41, pad=np.nan)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    say("bf16 wide spread")
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=3, refresh_cols=32, block=16, depth=8,
                       flags=lib.F_FORCE_GRID)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=3, refresh_cols=32)
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] > 245
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])


def test_bf16_wide_kernel_one_workgroup(lib):
    """The storage form on the single-workgroup wide-block kernel (a short
    wide system), with refreshes, against the oracle of the form."""
    rng = np.random.default_rng(43)
    s = gen.make_system(rng, 2000, 480, noise=0.01, pad=np.nan)
    X32 = dev(s.Xt)
    Xb = lib.convert_bf16(X32)
    say("bf16 wide one workgroup")
    r = lib.solve_bf16(Xb, X32, dev(s.y), max_sweeps=3, refresh_cols=160, block=16, depth=8)
    ref = oracle.solve_bf16_refresh(s.Xt, s.y, s.m, max_sweeps=3, refresh_cols=160)
    assert r.info["kernel_kind"] == 8 and r.info["team_wgs"] == 1
    assert r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
    assert np.all(np.abs(np.asarray(r.hist) - np.asarray(ref.hist)) <= 1e-5 * ref.hist[0])


def test_fp32_confirmed_relative_residual_stop(lib):
    """Plain single precision with refreshes takes the same FP64-confirmed
    relative-residual stop as the storage form: the stop lands where the
    oracle's does (the oracle refreshing from the same FP32 X), and the FP64
    final check is under tol."""
    s = gen.wide(m=2000, n=20_000, seed=5)
    tol, check, refresh = 1e-6, 512, 2048
    say("fp32 confirmed stop")
    r = lib.solve(dev(s.Xt), dev(s.y), max_sweeps=3, stop=lib.STOP_REL_RESID, tol=tol, check_cols=check,
                  refresh_cols=refresh, block=8)
    ref = oracle.solve(s.Xt, s.y, s.m, max_sweeps=3, stop=oracle.STOP_REL_RESID, tol=tol, check_cols=check,
                       Xt_refresh=s.Xt, refresh_cols=refresh)
    say("cols", r.info["cols_done"], ref.cols, "refreshes", r.info["refreshes"], ref.refreshes)
    assert ref.converged and r.info["converged"] == 1
    assert r.info["final_rel_resid"] < tol
    assert r.info["cols_done"] == ref.cols and r.info["refreshes"] == ref.refreshes
    assert rel(r.a.cpu().numpy(), ref.a) <= 1e-5
