"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This package only *describes problems*: grids, finite-difference stencil
coefficients of the PDEs, initial conditions, raw source samples, sample and
output times.  It contains none of the method's arithmetic (no compression, no
Krylov, no exponentials); both the HIP path and the oracle receive the same
float64 arrays from here.
"""
from .workloads import (  # noqa: F401
    Problem,
    BurgersProblem,
    ade_windows,
    grid,
    smooth_field,
    ade_coeffs,
    burgers_diffusion_coeffs,
    chebyshev_lobatto,
    uniform_samples,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_c4_subset,
    manufactured_ade,
    manufactured_burgers,
    sawtooth_wave,
    split_windows,
    c2_source,
    random_ade_problem,
)
