"""Plain FP64 CPU oracle of the LES momentum-residual assembly.

TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.  ``lesasm_oracle.c`` holds the arithmetic; this module
compiles it with gcc and wraps it with ctypes.
"""
from .oracle import (TERM_ALL, TERM_CONV, TERM_LITERAL, TERM_PRES, TERM_SGS, TERM_VISC,  # noqa: F401
                     assemble, assemble_threads, build, divergence, element_laplacian, element_residual, element_stress_residual,
                     element_volume,
                     filter_width, friction_velocity, gauss, load, lumped_mass, ngauss, nnode, shape, vreman,
                     wall_assemble, wall_law)
