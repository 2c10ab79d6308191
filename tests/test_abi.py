"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/hpscd.h declares, its struct layouts match the
header, and arguments are rejected before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpscd.h")


@pytest.fixture(scope="module")
def hp():
    from paper_2104_12570_amd import hpscd
    return hpscd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpscd_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(hp):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(hp._lib, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", hp.LIB_PATH], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}\b", nm), f"{name} not exported"


def test_struct_layouts_match_header(hp):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "hpscd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(hpscd_opts), sizeof(hpscd_info),
         sizeof(hpscd_sys), offsetof(hpscd_opts, tol), offsetof(hpscd_info, final_norm),
         offsetof(hpscd_info, total_ms), offsetof(hpscd_sys, tol), offsetof(hpscd_info, kernel_kind),
         offsetof(hpscd_opts, thr), offsetof(hpscd_opts, order), offsetof(hpscd_info, diverged),
         offsetof(hpscd_info, rel_grad), offsetof(hpscd_opts, spin_timeout_us));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(hp.Opts), ctypes.sizeof(hp.Info), ctypes.sizeof(hp.Sys),
                   hp.Opts.tol.offset, hp.Info.final_norm.offset, hp.Info.total_ms.offset, hp.Sys.tol.offset,
                   hp.Info.kernel_kind.offset, hp.Opts.thr.offset, hp.Opts.order.offset, hp.Info.diverged.offset,
                   hp.Info.rel_grad.offset, hp.Opts.spin_timeout_us.offset]


def test_version(hp):
    assert hp._lib.hpscd_version() == 2


@pytest.mark.parametrize("case,msg", [
    (dict(m=0), "m must be"),
    (dict(n=0), "n must be"),
    (dict(X=0), "X is NULL"),
    (dict(y=0), "y is NULL"),
    (dict(a=0), "a_out is NULL"),
    (dict(ldx=50), "ldx"),
    (dict(ldx=102), "multiple of 4"),
    (dict(X=8), "16-byte aligned"),
    (dict(elem=2, ldx=100), "multiple of 8"),
    (dict(max_sweeps=-1), "max_sweeps"),
    (dict(stop=7), "stop rule"),
    (dict(tol=float("nan")), "tol"),
    (dict(tol=-1.0), "tol"),
    (dict(block=3), "block"),
    (dict(block=64), "block"),
    (dict(block=32, depth=8), "chain kernel"),
    (dict(block=16, depth=5), "block 16"),
    (dict(block=8, depth=9), "chain kernel"),
    (dict(thr=4, depth=9), "wide-block kernel"),
    (dict(flags=2 | 4), "exclusive"),
    (dict(thr=-1), "thr"),
    (dict(thr=4, order=256), "exclusive"),
    (dict(thr=4, depth=5), "wide-block kernel"),
    (dict(order=256, depth=2), "wide-block kernel"),
    (dict(thr=4, block=8), "blocks of 16"),
    (dict(order=256, refresh=64), "refreshes"),
])
def test_validation_rejects(hp, case, msg):
    kw = dict(m=100, n=10, X=4096, ldx=100, elem=4, y=64, a=128, max_sweeps=5, stop=0, tol=0.0, block=0, flags=0,
              thr=0, order=0, depth=0, refresh=0)
    kw.update(case)
    o = hp.make_opts(kw["max_sweeps"], kw["stop"], kw["tol"], 0, kw["refresh"], kw["block"], kw["flags"],
                     depth=kw["depth"], thr=kw["thr"], order_ptr=kw["order"])
    st = hp.validate(kw["m"], kw["n"], kw["X"], kw["ldx"], kw["elem"], kw["y"], o, kw["a"])
    assert st == hp.EINVAL
    assert msg in hp.last_error()


def test_validation_accepts(hp):
    o = hp.make_opts(5)
    assert hp.validate(100, 10, 4096, 100, 4, 64, o, 128) == hp.OK
    assert hp.validate(100, 10, 4096, 104, 2, 64, o, 128) == hp.OK
    for kw in (dict(stop=hp.STOP_REL_GRAD, tol=1e-6), dict(thr=50), dict(thr=1, depth=5), dict(order_ptr=256),
               dict(thr=7, depth=8, block=16)):
        assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, **kw), 128) == hp.OK, kw


@pytest.mark.parametrize("depth", [0, 2, 3, 4, 5, 8, 9])
def test_kernel_kinds_accepted(hp, depth):
    o = hp.make_opts(5, depth=depth)
    assert hp.validate(100, 10, 4096, 100, 4, 64, o, 128) == hp.OK


@pytest.mark.parametrize("depth", [1, 6, 7, 10, 11, 12, 13, 14, -1])
def test_unknown_kernel_kind_rejected(hp, depth):
    o = hp.make_opts(5, depth=depth)
    assert hp.validate(100, 10, 4096, 100, 4, 64, o, 128) == hp.EINVAL
    assert "depth" in hp.last_error()


def test_null_context_rejected(hp):
    o = hp.make_opts(5)
    st = hp._lib.hpscd_solve_f32(None, 100, 10, 4096, 100, 64, None, ctypes.byref(o), 128, None, None, None)
    assert st == hp.EINVAL and "ctx" in hp.last_error()
    st = hp._lib.hpscd_solve_batched_f32(None, 0, None, 16, 16, None, ctypes.byref(o), 16, None, None, None,
                                         None, None, None)
    assert st == hp.EINVAL


def test_batch_validation(hp):
    o = hp.make_opts(5)
    table = hp._sys_array([[9000, 10, 0, 9000, 0, 0]])
    st = hp._lib.hpscd_solve_batched_f32(None, 1, table, 4096, 64, None, ctypes.byref(o), 128, None, None, None,
                                         None, None, None)
    assert st == hp.EINVAL and "exceeds" in hp.last_error()
    table = hp._sys_array([[100, 10, 2, 100, 0, 0]])
    st = hp._lib.hpscd_solve_batched_f32(None, 1, table, 4096, 64, None, ctypes.byref(o), 128, None, None, None,
                                         None, None, None)
    assert st == hp.EINVAL and "x_off" in hp.last_error()
    table = hp._sys_array([[100, 10, 0, 100, 0, 0]], tols=[-1.0])
    st = hp._lib.hpscd_solve_batched_f32(None, 1, table, 4096, 64, None, ctypes.byref(o), 128, None, None, None,
                                         None, None, None)
    assert st == hp.EINVAL and "tol" in hp.last_error()


def test_create_without_device(hp):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert hp._lib.hpscd_create(0, ctypes.byref(h)) == hp.EDEVICE


def test_single_hip_runtime_shared_with_torch(hp):
    """The library binds to the HIP runtime torch loaded (one runtime per process)."""
    import torch
    maps = hp.hip_runtimes_mapped()
    assert len(maps) == 1
    assert os.path.dirname(torch.__file__) in maps[0]


def test_mlp_create_rejects_bad_widths(hp):
    h = ctypes.c_void_p()
    assert hp._lib.hpscd_mlp_create(16, 13, 0, 256, 64, 0, ctypes.byref(h)) == hp.EINVAL
    assert "widths" in hp.last_error()
    assert hp._lib.hpscd_mlp_create(None, 13, 256, 256, 64, 0, ctypes.byref(h)) == hp.EINVAL
    assert "ctx" in hp.last_error()
    assert hp._lib.hpscd_mlp_create(16, 13, 256, 256, 64, 0, None) == hp.EINVAL
    assert hp._lib.hpscd_mlp_fit_output_scaling(None, 1, 16, None) == hp.EINVAL
    assert hp._lib.hpscd_mlp_num_params(None) == 0
    assert hp._lib.hpscd_mlp_forward(None, 1, 16, 16, None) == hp.EINVAL
    hp._lib.hpscd_mlp_destroy(None)


def test_batched_plan_rejects_bad_arguments(hp):
    o = hp.make_opts(5)
    h = ctypes.c_void_p()
    table = hp._sys_array([[100, 10, 0, 100, 0, 0]])
    assert hp._lib.hpscd_batched_plan_create(None, 1, table, 4096, 64, None, ctypes.byref(o), 128,
                                             ctypes.byref(h)) == hp.EINVAL
    assert "ctx" in hp.last_error()
    assert hp._lib.hpscd_batched_plan_create(None, 0, table, 4096, 64, None, ctypes.byref(o), 128,
                                             ctypes.byref(h)) == hp.EINVAL
    assert hp._lib.hpscd_batched_plan_launch(None, None) == hp.EINVAL
    assert hp._lib.hpscd_batched_plan_results(None, None, None, None, None, None, None) == hp.EINVAL
    hp._lib.hpscd_batched_plan_destroy(None)


def test_wide_block_needs_the_wide_kernel(hp):
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, block=16, depth=8), 128) == hp.OK
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, block=16), 128) == hp.OK
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, block=16, depth=5), 128) == hp.EINVAL
    assert "depth 8" in hp.last_error()


def test_spin_timeout_option(hp):
    """The bound on grid waits: 0 keeps the default, a negative bound is rejected."""
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, spin_timeout_us=0), 128) == hp.OK
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, spin_timeout_us=50), 128) == hp.OK
    assert hp.validate(100, 10, 4096, 100, 4, 64, hp.make_opts(5, spin_timeout_us=-1), 128) == hp.EINVAL
    assert "spin_timeout_us" in hp.last_error()


def test_select_rejects_bad_arguments(hp):
    J = (ctypes.c_int32 * 4)()
    cnt = ctypes.c_int32()
    args = dict(ctx=16, m=100, n=10, X=4096, ldx=100, y=64, a0=None, F=3, tol=0.0, a=128, J=J, cnt=ctypes.byref(cnt))

    def call(**kw):
        a = dict(args)
        a.update(kw)
        return hp._lib.hpscd_select_f32(a["ctx"], a["m"], a["n"], a["X"], a["ldx"], a["y"], a["a0"], a["F"],
                                        a["tol"], a["a"], a["J"], None, None, a["cnt"], None)

    for kw, msg in ((dict(ctx=None), "ctx"), (dict(m=0), "m and n"), (dict(X=None), "must not be NULL"),
                    (dict(J=None), "J_out"), (dict(ldx=98), "ldx"), (dict(X=4100), "ldx"), (dict(F=-1), "F must"),
                    (dict(tol=float("inf")), "tol"), (dict(tol=-0.5), "tol")):
        assert call(**kw) == hp.EINVAL, kw
        assert msg in hp.last_error(), (kw, hp.last_error())


def test_read_stream_rejects_bad_arguments(hp):
    ms = ctypes.c_double()
    assert hp._lib.hpscd_read_stream(None, 4096, 1024, 1, ctypes.byref(ms), None) == hp.EINVAL
    assert hp._lib.hpscd_read_stream(16, 4096, 1000, 1, ctypes.byref(ms), None) == hp.EINVAL
    assert "multiple of 16" in hp.last_error()
    assert hp._lib.hpscd_read_stream(16, 4100, 1024, 1, ctypes.byref(ms), None) == hp.EINVAL
    assert hp._lib.hpscd_read_stream(16, 4096, 1024, 0, ctypes.byref(ms), None) == hp.EINVAL
    assert "passes" in hp.last_error()
