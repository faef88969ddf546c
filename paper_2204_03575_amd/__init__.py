"""MI355X library for the per-time-step solve of the ternary Cahn-Hilliard model.

The computation lives in the HIP library ``libchm.so`` (C ABI in
``include/chm.h``); :mod:`paper_2204_03575_amd.chm` is its Python binding.
"""
from .chm import (ENTRY_POINTS, ChmError, Solver, chm_quadrature, library,  # noqa: F401
                  params_from_dict)
