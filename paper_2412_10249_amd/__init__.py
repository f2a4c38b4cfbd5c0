"""ImaSk (arXiv 2412.10249) hot path on AMD Instinct MI355X (gfx950).

The computation lives in libimask (HIP kernels behind the C ABI of
include/imask.h); this package marshals torch tensors and streams into it.
"""
from ._abi import (  # noqa: F401
    BUDGET_EPOCHS, BUDGET_ITERS, COMPENSATE, DRAW_COMMON, DRAW_INDEPENDENT, FULL_PAPER, FULL_UNBIASED, PROJECT, PROLONG,
    REG_SMOOTH_TV, REG_TIKHONOV, REG_TV, RESTRICT, RESTRICT_ADJ, SCHEDULE_PARALLEL, SCHEDULE_SEQUENTIAL, ImaskError,
    LIB_PATH, KERNEL_FORWARD, KERNEL_TRANSPOSE, KERNEL_TRANSPOSE_SUM,
)
from .imask import (  # noqa: F401
    Geometry, Levels, Params, Problem, Regularizer, backproject, block_draws, draws, project, resample,
    sigma_balamurugan, sigma_thm3, sketch_apply, step_constants, step_many, time_kernel, workspace,
)
