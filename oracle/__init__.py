"""CPU float64 oracle for AA-PDHG / FAA-PDHG.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and
by the CPU-baseline leg of bench.py.  The GPU library never imports, links or
runs anything here, and nothing here imports the GPU library.
"""
from .aapdhg_oracle import (  # noqa: F401
    ROW_EQ, ROW_GE, VARIANT_AA, VARIANT_FAA, VARIANT_PDHG, VARIANT_RPDHG, Options, Problem, Solver, State,
    aa_gamma, angle_filter, dhat, kkt, length_bounds, length_filter, pdhg_map, power_norm, power_start,
    splitmix64,
    pock_chambolle, proj_Lambda, proj_X, proj_Y, reverse, ruiz, solve)
