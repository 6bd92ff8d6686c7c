"""CPU oracle for the spkMC hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps ``liboracle_spkmc.so`` (plain C, see spkmc_oracle.c)
with ctypes and adds the L = 2 exact enumeration in ``enumerate2``.
"""
from .oracle import (  # noqa: F401
    Params, Record, Sim, Bkl, lib, philox, u53, uopen52, idx, rate_table, select,
    observables, site_class, init_spins, set_threads, get_threads,
)
