"""CPU FP64 oracle for the RGF hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy code written from the paper's statement of
the NEGF problem (Eqs. 1-8).  It shares no code with the HIP path and never
imports it.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path must never route through it.

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
from .negf_oracle import (  # noqa: F401
    fermi,
    norm1,
    sancho_rubio,
    lead_selfenergy,
    lead_lesser,
    rgf,
    dense,
    scba_selfenergy,
    scat_matrix,
    atom_blocks,
    solve_points,
    lead_tables,
    cap_selfenergy,
    scba,
    observables,
    dense_grad,
    density_objective,
)
from .poisson import (  # noqa: F401
    PoissonGrid,
    poisson_beta,
    poisson_matrix,
    poisson_boundary,
    density_atoms,
    density_jacobian,
    density_jacobian_local,
    newton_poisson,
)
