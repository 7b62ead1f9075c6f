"""Exact Gaussian-process regression on the AMD Instinct MI355X (gfx950).

The hot path (covariance assembly, tiled Cholesky, triangular solves,
posterior mean and variance, log marginal likelihood, its gradient and Adam
hyperparameter optimisation) runs in hand-written HIP kernels behind the
C-ABI of include/gpr.h; ``_lib`` is the ctypes binding and ``gp`` the
torch-facing front end (torch supplies device memory and streams only).
"""
from . import _lib
from ._lib import GprError, PRECISIONS

__all__ = ["_lib", "GprError", "PRECISIONS"]
