"""FP64 CPU oracle for the D3Q19 LBM of arXiv:1508.02960 (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It loads ``liblbm_oracle.so`` built from
``lbm_oracle.c`` (see :func:`build`) and shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    COLLISIONS, WALLS, Oracle, build, lattice, mrt_matrix, mrt_rates,
    trt_omega_minus, equilibrium, collide, collide_mrt_rates, voxelise,
    link_q, wall_q, library_path, set_threads,
)
