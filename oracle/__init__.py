"""FP64 CPU oracle of the repeated-pattern FETI method.  TEST INFRASTRUCTURE ONLY:
imported by the tests, the smoke check and the benchmark's CPU-baseline leg, never by the
GPU library or its binding."""
from .feti import (ETA_DROP, KERNEL_TAU, FetiOracle, PatternOracle, constrained_solve, global_solve, kernel_basis,
                   multipliers_from_displacements, pseudo_inverse)

__all__ = ["ETA_DROP", "KERNEL_TAU", "FetiOracle", "PatternOracle", "global_solve", "kernel_basis",
           "multipliers_from_displacements", "pseudo_inverse"]
