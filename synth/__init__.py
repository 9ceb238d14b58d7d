"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the discretisation or of the solver: it only
draws random numbers (SplitMix64), lays out mesh vertex coordinates and samples
the prescribed coefficient fields at given points.  Both the CPU oracle and the HIP
library receive the exact bytes produced here.
"""
from .splitmix import splitmix64_u64, uniform01, uniform_pm1, log_uniform
from .workloads import (unit_cube_vertices, perturbed_vertices, cell_coefficients,
                        rhs_values, multi_rhs, c5_alpha, reference_sample_points,
                        c5_coefficient_samples, batch_spec, WORKLOADS)

__all__ = ["splitmix64_u64", "uniform01", "uniform_pm1", "log_uniform",
           "unit_cube_vertices", "perturbed_vertices", "cell_coefficients",
           "rhs_values", "multi_rhs", "c5_alpha", "reference_sample_points",
           "c5_coefficient_samples", "batch_spec", "WORKLOADS"]
