"""Seeded synthetic workloads for the φ-combination solver.

This package only draws random inputs (coefficient fields, vectors, step sizes)
and describes the operators as plain data.  It holds none of the solver's or
the oracle's arithmetic, so both the HIP path and the CPU oracle can take their
inputs from it without sharing code.
"""

from .generators import (  # noqa: F401
    StencilDesc,
    CsrDesc,
    Problem,
    adr2d_problem,
    cfg1,
    cfg2,
    cfg2_tau_grid,
    cfg3,
    cfg4,
    cfg5_requests,
    diffusion3d_problem,
    csr_from_random_pattern,
    random_vectors,
    Request,
)
