"""MI355X (gfx950) vectorized-PSDP hot path: HIP kernels behind a C ABI.

The public functions forward to libpsdp.so through ``binding``; they raise if
the library is not built. Nothing here computes on the CPU.
"""
from .binding import (  # noqa: F401
    F32, F64, BF16, I8, PABB, PPA, EXIT_NAMES, PSDPError, Params, Stats,
    DIGIT_LAYOUTS, default_params, digit_choice, eval_penalty_grad, install_tuning, load, penalty_adjoint,
    penalty_fn, set_digit_table,
    perturbation, plan_columns, qx_dense, qx_digits, qx_single, round_objective, solve, solve_group, solve_host,
)
