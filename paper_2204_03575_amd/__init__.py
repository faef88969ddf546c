"""MI355X library for the per-time-step solve of the ternary Cahn-Hilliard model.

The computation lives in the HIP library ``libchm.so`` (C ABI in
``include/chm.h`` and ``include/chm_net.h``); :mod:`paper_2204_03575_amd.chm`
is its Python binding.
"""
from .chm import (ENTRY_POINTS, NET_NPARAMS, ChmError, Net, Solver, chm_quadrature,  # noqa: F401
                  flatten_params, library, params_from_dict, step_many, unflatten_params)
