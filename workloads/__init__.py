"""Seeded, synthetic problem data for the 2-D two-sided space-fractional diffusion equation.

This package only *describes problems*: grids, diffusion-coefficient fields, initial data,
manufactured exact solutions and their closed-form Riemann-Liouville source terms, and seeded
noise.  It contains none of the discretisation or solver arithmetic (no Grunwald weights, no
Toeplitz operators, no multigrid, no Krylov), so both the CPU oracle and the GPU library can take
their inputs from here without sharing any of the method's code.
"""
from .problems import (  # noqa: F401
    Problem,
    grid,
    sample,
    sample_u0,
    sample_source,
    source_terms,
    Request,
    random_instance,
    example1,
    example2,
    example3,
    config_c1,
    config_c2,
    config_c3,
    config_c4_instances,
    config_c5_requests,
    noise_field,
    poly_rl_left,
    poly_rl_right,
)
