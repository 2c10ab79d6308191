"""The allocation-free entry point (hpscd_solve_f32_noalloc) against
hpscd_solve_f32 through the C ABI: two calls in a row on the same device's
scratch area, the second on a smaller system, give the existing entry
point's results bit for bit (the same kernels on the same plan); a system
whose workspace exceeds the scratch area is refused before any device work.
"""
import ctypes

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _call(lib, name, s, Xt, y, a0, opts):
    import torch
    a = torch.empty(s.n, dtype=torch.float32, device="cuda")
    hist = np.full(opts.max_sweeps + 1, np.nan)
    info = lib.Info()
    st = getattr(lib._lib, name)(lib.context(), s.m, s.n, lib._ptr(Xt), Xt.shape[1], lib._ptr(y), lib._ptr(a0),
                                 ctypes.byref(opts), lib._ptr(a), hist.ctypes.data_as(lib._dp), ctypes.byref(info),
                                 lib._stream())
    torch.cuda.synchronize()
    return st, a.cpu().numpy(), hist, info.as_dict()


def _same(lib, s, a0=None, **kw):
    Xt, y = _dev(s.Xt), _dev(s.y)
    a0d = _dev(a0) if a0 is not None else None
    opts = lib.make_opts(**kw)
    st1, a1, h1, i1 = _call(lib, "hpscd_solve_f32_noalloc", s, Xt, y, a0d, opts)
    assert st1 == lib.OK, lib.last_error()
    st0, a0_, h0, i0 = _call(lib, "hpscd_solve_f32", s, Xt, y, a0d, opts)
    assert st0 == lib.OK, lib.last_error()
    assert np.array_equal(a1, a0_)
    assert np.array_equal(h1, h0, equal_nan=True)
    for k in ("sweeps_done", "converged", "cols_done", "zero_cols", "final_rel_resid", "final_norm", "block_used",
              "team_wgs", "kernel_kind", "diverged"):
        assert i1[k] == i0[k], (k, i1[k], i0[k])
    return i1


def test_noalloc_matches_solve_two_calls(lib):
    print("noalloc: 1M x 256, relative-change stop", flush=True)
    big = gen.tall_large()
    info = _same(lib, big, max_sweeps=100, stop=lib.STOP_REL_CHANGE, tol=1e-6)
    assert info["converged"] == 1 and info["team_wgs"] == 256
    print("noalloc: 2000 x 50 with a0 after the large call", flush=True)
    small = gen.tall_small(pad=np.nan)
    a0 = np.random.default_rng(3).standard_normal(small.n).astype(np.float32)
    info = _same(lib, small, a0=a0, max_sweeps=30, stop=lib.STOP_REL_CHANGE, tol=1e-9)
    assert info["sweeps_done"] >= 1
    # a variant of the method through the same area
    _same(lib, small, max_sweeps=8, thr=7)


def test_noalloc_refuses_a_workspace_beyond_the_scratch_area(lib):
    """Two million columns need more than the scratch area for their column
    statistics (reciprocal norms, in-block Gram entries, coefficients).  The
    refusal comes from the host before any launch (X is a small tensor here;
    nothing reads it)."""
    import torch
    X = torch.zeros(16, dtype=torch.float32, device="cuda")
    m, n = 2000, 2_000_000
    opts = lib.make_opts(max_sweeps=2)
    info = lib.Info()
    a = torch.zeros(16, dtype=torch.float32, device="cuda")
    st = lib._lib.hpscd_solve_f32_noalloc(lib.context(), m, n, lib._ptr(X), m, lib._ptr(X), None,
                                          ctypes.byref(opts), lib._ptr(a), None, ctypes.byref(info), lib._stream())
    assert st == lib.EINVAL and "scratch area" in lib.last_error()
