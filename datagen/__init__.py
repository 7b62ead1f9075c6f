"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the Gaussian-process method itself: it only
simulates the mass-spring-damper system whose lagged inputs are the regressors
(the paper's Section 5 workload), draws seeded random numbers and standardises
the columns.  Both the CPU oracle and the GPU path consume its output.
"""
from .msd import MSDConfig, simulate_msd, make_dataset, Dataset, subsample_indices, draw_c5_params

__all__ = ["MSDConfig", "simulate_msd", "make_dataset", "Dataset", "subsample_indices",
           "draw_c5_params"]
