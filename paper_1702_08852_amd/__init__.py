"""MI355X dual messenger Wiener filter: HIP library + thin Python binding.

The compute path is libdmwf.so (include/dmwf.h); `dmwf.Plan` marshals torch
tensors into it.  Importing this package does not load the library; the first
Plan does, and fails loudly if it was not built.
"""
from .dmwf import DmwfError, Plan, SolveStats, load, n_alm, status_string  # noqa: F401
