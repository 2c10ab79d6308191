"""Python binding of libhpscd (ctypes).

Argument marshalling only: every step of the solver runs in the HIP kernels
of ``libhpscd.so``.  PyTorch supplies device memory and the current stream.
Importing this module fails loudly when the library has not been built.

Layout: a system's X is passed as a torch tensor ``Xt`` of shape ``(n, ldx)``
(C-contiguous), i.e. column-major X with column j in ``Xt[j, :m]``.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np
# torch's HIP runtime must be loaded before the library: libhpscd.so then binds
# to that same runtime (same SONAME), so torch's allocations and stream handles
# are valid in every call.  Loading the library first would map a second HIP
# runtime into the process.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhpscd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2104_12570_amd.build` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)


def hip_runtimes_mapped():
    """Distinct HIP runtime files mapped into this process (expected: one)."""
    with open("/proc/self/maps") as f:
        return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})


if len(hip_runtimes_mapped()) != 1:
    raise ImportError(f"expected one HIP runtime in the process, found {hip_runtimes_mapped()}")

STOP_NONE, STOP_REL_CHANGE, STOP_REL_RESID, STOP_REL_GRAD = 0, 1, 2, 3
F_NO_FINAL_CHECK, F_FORCE_GRID, F_FORCE_WG, F_NO_COOP = 1, 2, 4, 8

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EABORTED, ETIMEOUT = range(7)
_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENONFINITE", 5: "EABORTED", 6: "ETIMEOUT"}


class Opts(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("stop", ctypes.c_int32), ("tol", ctypes.c_double),
                ("check_cols", ctypes.c_int64), ("refresh_cols", ctypes.c_int64), ("block", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("team_threads", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("thr", ctypes.c_int32), ("order", ctypes.c_void_p), ("spin_timeout_us", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int32), ("converged", ctypes.c_int32), ("cols_done", ctypes.c_int64),
                ("zero_cols", ctypes.c_int64), ("final_norm", ctypes.c_double),
                ("final_rel_resid", ctypes.c_double), ("y_norm", ctypes.c_double),
                ("block_used", ctypes.c_int32), ("team_wgs", ctypes.c_int32), ("team_threads", ctypes.c_int32),
                ("refreshes", ctypes.c_int32), ("sweep_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("kernel_kind", ctypes.c_int32), ("diverged", ctypes.c_int32), ("rel_grad", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Sys(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("x_off", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("y_off", ctypes.c_int64), ("a_off", ctypes.c_int64),
                ("tol", ctypes.c_double)]


_vp, _i64, _i32, _dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
_OP, _IP = ctypes.POINTER(Opts), ctypes.POINTER(Info)

_SIGS = {
    "hpscd_version": (ctypes.c_int, []),
    "hpscd_last_error": (ctypes.c_char_p, []),
    "hpscd_default_opts": (None, [_OP]),
    "hpscd_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "hpscd_destroy": (None, [_vp]),
    "hpscd_validate": (ctypes.c_int, [_i64, _i64, _vp, _i64, ctypes.c_int, _vp, _OP, _vp]),
    "hpscd_solve_f32": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _OP, _vp, _dp, _IP, _vp]),
    "hpscd_solve_f32_noalloc": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _OP, _vp, _dp, _IP, _vp]),
    "hpscd_solve_bf16": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _OP, _vp, _dp, _IP, _vp]),
    "hpscd_convert_bf16": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp]),
    "hpscd_residual_f64": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _dp, _vp]),
    "hpscd_solve_batched_f32": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Sys), _vp, _vp, _vp, _OP, _vp, _dp,
                                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                               _dp, _IP, _vp]),
    "hpscd_autotune_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Sys), _vp, _vp, _OP, _vp, _vp]),
    "hpscd_abort": (ctypes.c_int, [_vp]),
    "hpscd_read_stream": (ctypes.c_int, [_vp, _vp, _i64, _i32, _dp, _vp]),
    "hpscd_select_f32": (ctypes.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _i32, ctypes.c_double, _vp,
                                        ctypes.POINTER(ctypes.c_int32), _dp, _dp, ctypes.POINTER(ctypes.c_int32),
                                        _vp]),
    "hpscd_batched_plan_create": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(Sys), _vp, _vp, _vp, _OP, _vp,
                                                 ctypes.POINTER(_vp)]),
    "hpscd_batched_plan_launch": (ctypes.c_int, [_vp, _vp]),
    "hpscd_batched_plan_results": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int32),
                                                  ctypes.POINTER(ctypes.c_int32), _dp, _IP, _vp]),
    "hpscd_batched_plan_destroy": (None, [_vp]),
    "hpscd_mlp_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "hpscd_mlp_destroy": (None, [_vp]),
    "hpscd_mlp_num_params": (_i64, [_vp]),
    "hpscd_mlp_set_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "hpscd_mlp_get_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "hpscd_mlp_forward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "hpscd_mlp_grads": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_float), _vp]),
    "hpscd_mlp_train_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_float), _vp]),
    "hpscd_mlp_fit_output_scaling": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "hpscd_mlp_get_output_scaling": (ctypes.c_int, [_vp, _vp, _vp]),
    "hpscd_mlp_set_output_scaling": (ctypes.c_int, [_vp, _vp, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class HPSCDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st):
    if st != OK:
        raise HPSCDError(st, _lib.hpscd_last_error().decode())


def last_error() -> str:
    return _lib.hpscd_last_error().decode()


def make_opts(max_sweeps=100, stop=STOP_NONE, tol=0.0, check_cols=0, refresh_cols=0, block=0, flags=0,
              team_threads=0, depth=0, thr=0, order_ptr=0, spin_timeout_us=0) -> Opts:
    o = Opts()
    _lib.hpscd_default_opts(ctypes.byref(o))
    o.max_sweeps, o.stop, o.tol = int(max_sweeps), int(stop), float(tol)
    o.check_cols, o.refresh_cols, o.block, o.flags = int(check_cols), int(refresh_cols), int(block), int(flags)
    o.team_threads = int(team_threads)
    o.depth = int(depth)
    o.thr = int(thr)
    o.order = int(order_ptr) or None
    o.spin_timeout_us = int(spin_timeout_us)
    return o


def validate(m, n, X_ptr, ldx, elem_bytes, y_ptr, opts: Opts, a_ptr) -> int:
    """Host-only argument check (no device needed); returns the status code."""
    return _lib.hpscd_validate(m, n, X_ptr, ldx, elem_bytes, y_ptr, ctypes.byref(opts), a_ptr)


# --------------------------------------------------------------- device side
_CTX = {}
_LIVE = weakref.WeakSet()   # plans and networks still holding library objects
_SHUTDOWN = False


def _shutdown():
    """Release every library object while the HIP runtime (and a profiler
    wrapped around the process) is still fully up: Python's atexit hooks run
    before the interpreter tears modules down and before the C runtime's own
    exit handlers, where the runtime and any tool attached to it finalise.
    Objects collected later find the flag set and release nothing."""
    global _SHUTDOWN
    if _SHUTDOWN:
        return
    _SHUTDOWN = True
    try:
        torch = _torch()
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass
    for dev in list(_CTX):
        _lib.hpscd_destroy(_CTX.pop(dev))


atexit.register(_shutdown)


def _torch():
    import torch
    return torch


def context(device: int | None = None):
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _CTX:
        h = _vp()
        _check(_lib.hpscd_create(dev, ctypes.byref(h)))
        _CTX[dev] = h
    return _CTX[dev]


def _stream():
    return _vp(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _need_cuda(t, name, dtype=None):
    torch = _torch()
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class Result:
    a: object          # torch tensor (n,) float32
    hist: np.ndarray   # ||e|| after sweeps 0..sweeps_done
    info: dict


def solve(Xt, y, a0=None, *, max_sweeps=100, stop=STOP_NONE, tol=0.0, check_cols=0, block=0, flags=0,
          team_threads=0, depth=0, want_hist=True, thr=0, order=None, refresh_cols=0,
          spin_timeout_us=0) -> Result:
    """Solve X·a = y (Algorithm 1, single precision) on the GPU.

    Xt: (n, ldx) float32 CUDA tensor (column j of X in Xt[j, :m]); y: (m,).
    thr > 1: the parallel solver (Algorithm 2) with blocks of thr columns.
    order: None (cyclic) or an int32 CUDA tensor (>= max_sweeps, n) whose
    row s-1 lists the columns of sweep s.  spin_timeout_us: bound on every
    wait of a grid's workgroups for one another (0 = 10 s); past it the
    call raises HPSCDError with status ETIMEOUT."""
    torch = _torch()
    _need_cuda(Xt, "Xt", torch.float32)
    _need_cuda(y, "y", torch.float32)
    _need_cuda(a0, "a0", torch.float32)
    n, ldx = Xt.shape
    m = y.numel()
    if order is not None:
        _need_cuda(order, "order", torch.int32)
        if order.dim() != 2 or order.shape[1] != n or order.shape[0] < max_sweeps:
            raise ValueError("order must have shape (>= max_sweeps, n)")
    a = torch.empty(n, dtype=torch.float32, device=Xt.device)
    opts = make_opts(max_sweeps, stop, tol, check_cols, refresh_cols, block, flags, team_threads, depth, thr,
                     order.data_ptr() if order is not None else 0, spin_timeout_us)
    hist = np.full(max_sweeps + 1, np.nan) if want_hist else None
    info = Info()
    _check(_lib.hpscd_solve_f32(context(Xt.device.index), m, n, _ptr(Xt), ldx, _ptr(y), _ptr(a0),
                                ctypes.byref(opts), _ptr(a),
                                hist.ctypes.data_as(_dp) if hist is not None else None,
                                ctypes.byref(info), _stream()))
    h = hist[: info.sweeps_done + 1] if hist is not None else None
    return Result(a, h, info.as_dict())


@dataclass
class SelectResult:
    a: object          # torch tensor (n,) float32: a0 plus the selected steps
    J: list            # selected columns, in order
    da: np.ndarray     # step taken for each selected column
    hist: np.ndarray   # ||e|| before the first and after each selection
    count: int


def select(Xt, y, F, a0=None, *, tol=0.0) -> SelectResult:
    """Feature selection with HPSCD (Algorithm 3) on the GPU: F greedy
    choices of the column whose one-column step lowers ||e|| most."""
    torch = _torch()
    _need_cuda(Xt, "Xt", torch.float32)
    _need_cuda(y, "y", torch.float32)
    _need_cuda(a0, "a0", torch.float32)
    n, ldx = Xt.shape
    m = y.numel()
    F = int(F)
    a = torch.empty(n, dtype=torch.float32, device=Xt.device)
    J = np.full(max(F, 1), -1, np.int32)
    da = np.full(max(F, 1), np.nan)
    hist = np.full(F + 1, np.nan)
    cnt = ctypes.c_int32()
    _check(_lib.hpscd_select_f32(context(Xt.device.index), m, n, _ptr(Xt), ldx, _ptr(y), _ptr(a0), F, float(tol),
                                 _ptr(a), J.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), da.ctypes.data_as(_dp),
                                 hist.ctypes.data_as(_dp), ctypes.byref(cnt), _stream()))
    c = cnt.value
    return SelectResult(a, [int(j) for j in J[:c]], da[:c].copy(), hist[: c + 1].copy(), c)


def convert_bf16(Xt):
    """bfloat16 copy of X (round to nearest even), shape (n, ldx rounded up to 8)."""
    torch = _torch()
    _need_cuda(Xt, "Xt", torch.float32)
    n, ldx = Xt.shape
    ldd = (ldx + 7) // 8 * 8
    out = torch.empty((n, ldd), dtype=torch.bfloat16, device=Xt.device)
    _check(_lib.hpscd_convert_bf16(context(Xt.device.index), ldx, n, _ptr(Xt), ldx, _ptr(out), ldd, _stream()))
    return out


def solve_bf16(Xb, Xt32, y, a0=None, *, max_sweeps=100, stop=STOP_NONE, tol=0.0, check_cols=0, refresh_cols=0,
               block=0, flags=0, team_threads=0, depth=0, want_hist=True) -> Result:
    """bfloat16-storage form: sweeps read Xb, refreshes and the final check read Xt32."""
    torch = _torch()
    _need_cuda(Xb, "Xb", torch.bfloat16)
    _need_cuda(Xt32, "Xt32", torch.float32)
    _need_cuda(y, "y", torch.float32)
    _need_cuda(a0, "a0", torch.float32)
    n, ldxb = Xb.shape
    ldx = Xt32.shape[1]
    m = y.numel()
    a = torch.empty(n, dtype=torch.float32, device=Xb.device)
    opts = make_opts(max_sweeps, stop, tol, check_cols, refresh_cols, block, flags, team_threads, depth)
    hist = np.full(max_sweeps + 1, np.nan) if want_hist else None
    info = Info()
    _check(_lib.hpscd_solve_bf16(context(Xb.device.index), m, n, _ptr(Xb), ldxb, _ptr(Xt32), ldx, _ptr(y),
                                 _ptr(a0), ctypes.byref(opts), _ptr(a),
                                 hist.ctypes.data_as(_dp) if hist is not None else None,
                                 ctypes.byref(info), _stream()))
    h = hist[: info.sweeps_done + 1] if hist is not None else None
    return Result(a, h, info.as_dict())


def residual_f64(Xt, y, a, want_e=False):
    """r = y - X·a with FP64 sums; returns (||r||_2, r as float32 or None)."""
    torch = _torch()
    _need_cuda(Xt, "Xt", torch.float32)
    n, ldx = Xt.shape
    m = y.numel()
    e = torch.empty(m, dtype=torch.float32, device=Xt.device) if want_e else None
    nrm = ctypes.c_double()
    _check(_lib.hpscd_residual_f64(context(Xt.device.index), m, n, _ptr(Xt), ldx, _ptr(y), _ptr(a), _ptr(e),
                                   ctypes.byref(nrm), _stream()))
    return nrm.value, e


_SYS_DTYPE = np.dtype([("m", "<i8"), ("n", "<i8"), ("x_off", "<i8"), ("ldx", "<i8"), ("y_off", "<i8"),
                       ("a_off", "<i8"), ("tol", "<f8")])


class _SysTable:
    """hpscd_sys rows in a NumPy buffer, passed to C by address."""

    def __init__(self, rec):
        self.rec = rec

    @property
    def _as_parameter_(self):
        return ctypes.cast(self.rec.ctypes.data, ctypes.POINTER(Sys))

    def __getitem__(self, i):
        return Sys(*[v.item() for v in self.rec[i]])


def _sys_array(table, tols=None):
    """hpscd_sys table from rows (m, n, x_off, ldx, y_off, a_off) and optional
    per-system tolerances (0 = the call's tol)."""
    assert ctypes.sizeof(Sys) == _SYS_DTYPE.itemsize
    table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
    tols = np.zeros(len(table)) if tols is None else np.asarray(tols, dtype=np.float64).reshape(-1)
    if len(tols) != len(table):
        raise ValueError("tols needs one entry per system")
    rec = np.empty(len(table), dtype=_SYS_DTYPE)
    for k, name in enumerate(_SYS_DTYPE.names[:6]):
        rec[name] = table[:, k]
    rec["tol"] = tols
    return _SysTable(rec)


@dataclass
class BatchResult:
    a: object
    hist: np.ndarray | None
    sweeps: np.ndarray
    converged: np.ndarray
    final_rel_resid: np.ndarray
    info: dict


def solve_batched(Xpool, ypool, table, a0pool=None, *, max_sweeps=100, stop=STOP_NONE, tol=0.0, block=0,
                  flags=0, a_size=None, want_hist=False, tols=None, team_threads=0) -> BatchResult:
    """Solve every system of a packed batch in one persistent launch.
    ``table[i] = (m, n, x_off, ldx, y_off, a_off)``; ``tols[i] > 0`` replaces
    ``tol`` for system i."""
    torch = _torch()
    _need_cuda(Xpool, "Xpool", torch.float32)
    _need_cuda(ypool, "ypool", torch.float32)
    _need_cuda(a0pool, "a0pool", torch.float32)
    table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
    count = len(table)
    if a_size is None:
        a_size = int((table[:, 5] + table[:, 1]).max())
    a = torch.zeros(a_size, dtype=torch.float32, device=Xpool.device)
    opts = make_opts(max_sweeps, stop, tol, 0, 0, block, flags, team_threads)
    hist = np.full((count, max_sweeps + 1), np.nan) if want_hist else None
    sw = np.zeros(count, np.int32)
    cv = np.zeros(count, np.int32)
    fr = np.zeros(count)
    info = Info()
    _check(_lib.hpscd_solve_batched_f32(
        context(Xpool.device.index), count, _sys_array(table, tols), _ptr(Xpool), _ptr(ypool), _ptr(a0pool),
        ctypes.byref(opts), _ptr(a), hist.ctypes.data_as(_dp) if hist is not None else None,
        sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        fr.ctypes.data_as(_dp), ctypes.byref(info), _stream()))
    return BatchResult(a, hist, sw, cv, fr, info.as_dict())


class BatchPlan:
    """A batched solve recorded once as a HIP graph and replayed.  The pools
    are bound by address (keep the tensors alive; their contents may change
    between launches).  ``launch()`` queues a replay on the current stream;
    ``results()`` waits and returns a BatchResult (info times are NaN)."""

    def __init__(self, Xpool, ypool, table, a0pool=None, apool=None, *, max_sweeps=100, stop=STOP_NONE, tol=0.0,
                 block=0, flags=0, tols=None):
        torch = _torch()
        _need_cuda(Xpool, "Xpool", torch.float32)
        _need_cuda(ypool, "ypool", torch.float32)
        _need_cuda(a0pool, "a0pool", torch.float32)
        table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
        self.count = len(table)
        a_size = int((table[:, 5] + table[:, 1]).max())
        self.a = apool if apool is not None else torch.zeros(a_size, dtype=torch.float32, device=Xpool.device)
        _need_cuda(self.a, "apool", torch.float32)
        self._keep = (Xpool, ypool, a0pool, self.a)
        self.max_sweeps = int(max_sweeps)
        opts = make_opts(max_sweeps, stop, tol, 0, 0, block, flags)
        h = _vp()
        self._ctx = context(Xpool.device.index)
        _check(_lib.hpscd_batched_plan_create(self._ctx, self.count, _sys_array(table, tols), _ptr(Xpool),
                                              _ptr(ypool), _ptr(a0pool), ctypes.byref(opts), _ptr(self.a),
                                              ctypes.byref(h)))
        self._h = h
        _LIVE.add(self)

    def launch(self):
        _check(_lib.hpscd_batched_plan_launch(self._h, _stream()))

    def results(self, want_hist=False) -> BatchResult:
        hist = np.full((self.count, self.max_sweeps + 1), np.nan) if want_hist else None
        sw = np.zeros(self.count, np.int32)
        cv = np.zeros(self.count, np.int32)
        fr = np.zeros(self.count)
        info = Info()
        _check(_lib.hpscd_batched_plan_results(
            self._h, hist.ctypes.data_as(_dp) if hist is not None else None,
            sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            fr.ctypes.data_as(_dp), ctypes.byref(info), _stream()))
        return BatchResult(self.a, hist, sw, cv, fr, info.as_dict())

    def close(self):
        if getattr(self, "_h", None):
            _lib.hpscd_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        if _SHUTDOWN:
            return
        try:
            self.close()
        except Exception:
            pass


def autotune_batched(Xpool, ypool, table, *, max_sweeps=100, stop=STOP_NONE, tol=0.0, a_size=None):
    torch = _torch()
    table = np.asarray(table, dtype=np.int64).reshape(-1, 6)
    if a_size is None:
        a_size = int((table[:, 5] + table[:, 1]).max())
    a = torch.zeros(a_size, dtype=torch.float32, device=Xpool.device)
    opts = make_opts(max_sweeps, stop, tol)
    _check(_lib.hpscd_autotune_batched(context(Xpool.device.index), len(table), _sys_array(table), _ptr(Xpool),
                                       _ptr(ypool), ctypes.byref(opts), _ptr(a), _stream()))


def read_stream_ms(t, passes=10) -> float:
    """Device milliseconds of one pass of 16-byte loads over the bytes of the
    CUDA tensor t (the measured read-stream rate of HBM)."""
    ms = ctypes.c_double()
    nbytes = t.numel() * t.element_size() // 16 * 16
    _check(_lib.hpscd_read_stream(context(t.device.index), _ptr(t), nbytes, int(passes), ctypes.byref(ms), _stream()))
    return ms.value


def abort(device: int | None = None):
    _check(_lib.hpscd_abort(context(device)))


# ------------------------------------------------------------------ MLP
class MLP:
    """Handle of a device-resident perceptron in -> h1 -> h2 -> out (exact
    GELU on the hidden layers, linear output) with its Adam state.  All
    arithmetic runs in the library's kernels; tensors are FP32 on the device."""

    def __init__(self, n_in, h1, h2, n_out, device: int | None = None, seed: int = 0):
        torch = _torch()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.shape = (int(n_in), int(h1), int(h2), int(n_out))
        h = _vp()
        _check(_lib.hpscd_mlp_create(context(self.device), *self.shape, int(seed) & (2 ** 64 - 1), ctypes.byref(h)))
        self._h = h
        self.num_params = int(_lib.hpscd_mlp_num_params(h))
        _LIVE.add(self)

    def close(self):
        if getattr(self, "_h", None):
            _lib.hpscd_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        if _SHUTDOWN:
            return
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, name, width):
        torch = _torch()
        _need_cuda(t, name, torch.float32)
        if t.dim() != 2 or t.shape[1] != width:
            raise ValueError(f"{name} must have shape (batch, {width})")
        return t

    def set_params(self, flat):
        torch = _torch()
        _need_cuda(flat, "flat", torch.float32)
        if flat.numel() != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters")
        _check(_lib.hpscd_mlp_set_params(self._h, _ptr(flat), _stream()))

    def fit_output_scaling(self, targets):
        """Standardise the outputs by the per-output mean and sample standard
        deviation of ``targets`` (count, n_out): see hpscd.h."""
        targets = self._vec(targets, "targets", self.shape[3])
        _check(_lib.hpscd_mlp_fit_output_scaling(self._h, targets.shape[0], _ptr(targets), _stream()))

    def output_scaling(self):
        """(2 * n_out,) device tensor [mu..., sd...]."""
        torch = _torch()
        t = torch.empty(2 * self.shape[3], dtype=torch.float32, device=f"cuda:{self.device}")
        _check(_lib.hpscd_mlp_get_output_scaling(self._h, _ptr(t), _stream()))
        return t

    def set_output_scaling(self, mu_sd):
        torch = _torch()
        _need_cuda(mu_sd, "mu_sd", torch.float32)
        if mu_sd.numel() != 2 * self.shape[3]:
            raise ValueError(f"expected {2 * self.shape[3]} values")
        _check(_lib.hpscd_mlp_set_output_scaling(self._h, _ptr(mu_sd), _stream()))

    def get_params(self):
        torch = _torch()
        flat = torch.empty(self.num_params, dtype=torch.float32, device=f"cuda:{self.device}")
        _check(_lib.hpscd_mlp_get_params(self._h, _ptr(flat), _stream()))
        return flat

    def forward(self, x, out=None):
        torch = _torch()
        x = self._vec(x, "x", self.shape[0])
        y = torch.empty(x.shape[0], self.shape[3], dtype=torch.float32, device=x.device) if out is None else out
        _need_cuda(y, "out", torch.float32)
        if y.numel() != x.shape[0] * self.shape[3]:
            raise ValueError("out must hold batch * n_out values")
        _check(_lib.hpscd_mlp_forward(self._h, x.shape[0], _ptr(x), _ptr(y), _stream()))
        return y

    def grads(self, x, target):
        torch = _torch()
        x = self._vec(x, "x", self.shape[0])
        target = self._vec(target, "target", self.shape[3])
        g = torch.empty(self.num_params, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        _check(_lib.hpscd_mlp_grads(self._h, x.shape[0], _ptr(x), _ptr(target), _ptr(g), ctypes.byref(loss),
                                    _stream()))
        return g, loss.value

    def train_step(self, x, target, lr, want_loss=False):
        x = self._vec(x, "x", self.shape[0])
        target = self._vec(target, "target", self.shape[3])
        loss = ctypes.c_float()
        _check(_lib.hpscd_mlp_train_step(self._h, x.shape[0], _ptr(x), _ptr(target), float(lr),
                                         ctypes.byref(loss) if want_loss else None, _stream()))
        return loss.value if want_loss else None
