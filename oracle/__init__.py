"""CPU oracle (TEST INFRASTRUCTURE ONLY).

A plain FP64 C implementation of the ternary Cahn-Hilliard time step
(``chm_oracle.c``) and its ctypes wrapper.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may use it; the GPU library never
imports, links or calls it.
"""
from .oracle import Oracle, OracleError, build_oracle, oracle_params, load_library  # noqa: F401
