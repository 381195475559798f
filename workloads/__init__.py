"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This package generates *inputs* only: symmetric positive definite quadratic
problems 1/2 m^T A m - b^T m, the (s_i, y_i) pairs an optimizer produces on
them, and blocks of probe vectors.  It holds none of the BFGS, randomized-SVD
or posterior-variance arithmetic; both the GPU library and the CPU oracle
consume what it produces.
"""
from .quadratic import (  # noqa: F401
    GridQuadratic,
    DenseQuadratic,
    make_problem,
    cg_pairs,
    random_secant_pairs,
    normal_block,
    CONFIGS,
)
