"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

Contents
  mg_oracle.c   plain C: operator, right-hand side, CG, lexicographic
                Gauss-Seidel V-cycle (built into liboracle.so by build.py)
  oracle.py     ctypes front end + a pure-Python dense assembly for tiny grids
  nn_oracle.py  FP64 NumPy forward/backward of the 3D conv network layers
  amr_oracle.py the composite (base grid + refined patches) problem, assembled
                cell by cell and solved by a sparse direct solver
"""
from .oracle import (  # noqa: F401
    build,
    apply,
    rhs,
    residual,
    solve_cg,
    solve_vcycle,
    rbgs,
    rbgs_level,
    level_dims,
    prolong_add,
    solve_reference,
    dense_matrix,
    dense_solve,
    num_levels,
    threads,
    tga_coefficients,
    tga_step,
    field,
    relaxation_time,
)
