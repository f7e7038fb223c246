"""CPU FP64 oracle for the block-step Hermite N-body hot path.

Test infrastructure only: the tests, the package smoke check and the
benchmark's CPU-baseline leg use it; the product path never does.  It shares
no code with the HIP library (see ``nbody_oracle.c`` for the formulas and the
passages of the method they follow).
"""
from .oracle import (  # noqa: F401
    OracleConfig,
    build,
    lib_path,
    force,
    force_nb,
    pn_rel,
    pn_rel_derivs,
    pn,
    predict,
    hermite_high,
    hermite_correct,
    dt_crit,
    new_level,
    init,
    block_step,
    integrate,
    energy,
    num_threads,
    State,
)
