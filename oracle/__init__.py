"""CPU oracle for the HPSCD solver and its learned warm start.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
Plain NumPy in FP64, written from the paper's Algorithms 1-3 (Sections 2-3,
7 and 8);
see the module docstrings for the passage each function follows.
``mlp_oracle`` is the FP64 reference of the warm-start perceptron.
"""
from .hpscd_oracle import (  # noqa: F401
    STOP_NONE, STOP_REL_CHANGE, STOP_REL_RESID, STOP_REL_GRAD, OracleResult,
    SelectResult, residual, gradient, final_rel_resid, bf16_round, solve,
    solve_bf16_refresh, solve_batch, solve_parallel, select_features,
)
from . import mlp_oracle  # noqa: F401,E402
