"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the method itself: only the
counter-based normal generator that draws the KL coefficients xi, and the
workload definitions (grid sizes, field parameters, sample counts, seeds).
"""
from .xi import splitmix64_normals, xi_index_limits  # noqa: F401
from .workloads import WORKLOADS, workload, level_cells  # noqa: F401
