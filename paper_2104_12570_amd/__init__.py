"""MI355X (gfx950) implementation of the HPSCD column-wise solver for X·a = y.

The compute path is ``libhpscd.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/hpscd.h``); ``paper_2104_12570_amd.hpscd`` is its ctypes
binding.  The binding is imported lazily so that ``python -m
paper_2104_12570_amd.build`` works before the library exists.
"""

__all__ = ["hpscd", "warmstart"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
