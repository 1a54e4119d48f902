"""MI355X (gfx950) Gaussian belief propagation solver for A x = b.

Thin Python binding over the C ABI of ``libgabp.so`` (declared in
``include/gabp.h``).  Every function here only marshals arguments: device
tensors become raw pointers, the current torch stream becomes the HIP stream,
and the C status codes come back unchanged.  All arithmetic runs in the HIP
kernels of the library; there is no CPU fallback, and importing this package
fails if the library has not been built.
"""
from ._abi import (  # noqa: F401
    GABP_OK, GABP_NOT_CONVERGED, GABP_ERR_ARG, GABP_ERR_NOT_SYMMETRIC, GABP_ERR_ZERO_DIAG,
    GABP_ERR_BREAKDOWN, GABP_ERR_DIVERGED, GABP_ERR_HIP, GABP_ERR_NOMEM, GABP_ERR_UNSUPPORTED,
    GABP_LAYOUT_PAIR, GABP_LAYOUT_GATHER, GABP_SCHEDULE_SYNC, GABP_SCHEDULE_COLORED,
    LIB_PATH, DeviceCSR, GabpError, Opts, Stats, lib, status_name,
    gabp_default_opts, gabp_solve, gabp_residual, gabp_residual_noalloc, gabp_plan_create,
    gabp_plan_destroy,
    gabp_plan_solve, gabp_plan_reset, gabp_plan_sweeps, gabp_plan_marginals,
    gabp_plan_get_messages, gabp_plan_set_messages, gabp_version,
    DeviceGrid, gabp_plan_create_grid, gabp_solve_grid, gabp_residual_grid,
    GABP_BATCH_BIPARTITE, GABP_BATCH_DENSE, GABP_BATCH_CSR, DeviceBatch,
    GABP_ACCEL_NONE, GABP_ACCEL_AITKEN, GABP_ACCEL_STEFFENSEN,
    gabp_plan_create_batched, gabp_plan_solve_batched, gabp_solve_batched,
    GABP_MODEL_INPUTS, GABP_MODEL_OUTPUTS, GABP_MODEL_PARAMS, Model,
    gabp_model_create, gabp_model_get_params, gabp_model_set_params, gabp_model_forward,
    gabp_model_grad, gabp_model_train_step, gabp_model_grid_features, gabp_model_grid_targets,
    gabp_plan_solve_warm, gabp_plan_solve_coarse,
    gabp_plan_colors, DeviceRect, gabp_plan_create_lsq, gabp_plan_solve_lsq, gabp_solve_lsq,
    gabp_plan_residual_lsq, gabp_plan_workspace_bytes,
)
