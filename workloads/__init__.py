"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package draws random numbers and lays out arrays; it holds none of the
solver's arithmetic.  See ``workloads.gen``.
"""
from .gen import *  # noqa: F401,F403
