"""MI355X dual messenger Wiener filter: HIP library + thin Python binding.

The compute path is libdmwf.so (include/dmwf.h); `dmwf.Plan` marshals torch
tensors into it.  Importing this package does not load the library; the first
Plan does, and fails loudly if it was not built.
"""
from .dmwf import (BF16X3_GEMM, FP32_GEMM, FP64, DmwfError, Net, Plan, SolveStats,  # noqa: F401
                   load, n_alm, nn_features, noise_stats, solve_plans, status_string)
