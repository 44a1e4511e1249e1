"""Seeded synthetic problem generators shared by the oracle, the tests and the bench.

This package builds the linear systems A x = b that the solver is run on (the
2-D 5-point Laplace problem of the paper's experimental section, 3-D 7-point
and variable-coefficient finite-volume analogues) and their right-hand sides.
It holds none of the Schwarz method's arithmetic: no partitioning, overlap,
local solve or iteration lives here.
"""
from .problems import (
    CSR,
    laplace2d,
    laplace3d,
    tpfa2d,
    tpfa3d,
    gaussian_random_field_2d,
    uniform_rhs,
    manufactured_rhs,
    sine_mode_2d,
    sine_mode_3d,
    config_problem,
    serving_stream,
    serving_system,
    CONFIGS,
)

__all__ = [
    "CSR",
    "laplace2d",
    "laplace3d",
    "tpfa2d",
    "tpfa3d",
    "gaussian_random_field_2d",
    "uniform_rhs",
    "manufactured_rhs",
    "sine_mode_2d",
    "sine_mode_3d",
    "config_problem",
    "serving_stream",
    "serving_system",
    "CONFIGS",
]
