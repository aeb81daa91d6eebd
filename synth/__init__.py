"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only draws and lays out input arrays (grids, permittivity maps,
sources, boundary values).  It holds none of the solver's arithmetic: no
operator, no residual, no multigrid step.  Both the oracle and the GPU path
receive the same arrays from here and nothing else.
"""
from .problems import (  # noqa: F401
    Problem,
    manufactured_poisson,
    filament_source,
    streamer_set,
    batch_dims,
    random_problem,
    random_faces,
    diffusion_faces,
    HELMHOLTZ_KDX,
    TGA_DIFFUSION_NUMBER,
)
