"""Plain FP64 CPU oracle for exact Gaussian-process regression (test infrastructure).

This package is test infrastructure only: the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP path and imports nothing from it.

Every function states the passage of the paper (or the stated reading of it)
that it follows; floating point is float64 throughout (the paper uses double
precision BLAS, Section 5).
"""
from .gp import (LOG2PI, KERNELS, Hyper, sq_dist, se_cov, matern_of_r2, cov, dcov_dlog_ell, train_cov, cholesky, potrf_info, solve_alpha,
                 predict_mean, predict_var, nlml, nlml_grad, fit, adam_step, optimize,
                 cholesky_flops, tile_task_census)
from .mlp import (MLP_SIZES, mlp_init, mlp_unpack, mlp_forward, mlp_loss_and_grad, mlp_adam_step,
                  gelu, N_PARAMS)
from .stats import summary_stats, N_STATS
from .mixed import bf16_rne, split_bf16x3

__all__ = [n for n in dir() if not n.startswith("_")]
