"""Plain FP64 CPU oracle for the complex additive multilevel Helmholtz cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything under this directory; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path: its
only common dependency is the seeded input generator module, which holds none
of the method's arithmetic.

Everything here is written for clarity, not speed: numpy in complex128, the
operator assembled cell by cell from the 2^d x 2^d element matrices (the
paper's Appendix B element-wise matrix-free evaluation), the grid transfers as
tensor products of explicit 1D interpolation matrices, and the cycles as the
paper states them (Algorithm 1 "add", the appendix bottom-up FAS "buFAS", and
the single-sweep pipelined Algorithms tdAdd / tdBPX with the hb relaxation
mask of Section 5.2).

Parity status of each function is stated in its docstring; "pinned" names the
independent test that fixes it (closed form, textbook routine, brute force).
"""

from .discretisation import (  # noqa: F401
    element_matrices, level_eta, cell_theta, cell_eta, apply_H, diag_H, cell_average, coarse_fields,
    lumped_rhs, dense_H, norm_h, norm_max, zero_boundary, interior_mask,
)
from .transfer import prolong, restrict, inject, cpoint_mask, prolong_matrix_1d  # noqa: F401
from .cycle import (  # noqa: F401
    Params, omega_levels, semantic_cycle, textbook_additive, bottom_up_fas,
    Pipelined, zero_start_cycle,
)
from .solve import stationary_solve, bicgstab, dense_solve, nested_initial_guess, max_norm_reduction  # noqa: F401
from .adjoint import shell_functional, potential_gradient  # noqa: F401
