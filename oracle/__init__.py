"""FP64 CPU oracle for the near-field force (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    OracleError,
    build,
    lib_path,
    cells,
    bin_particles,
    accel,
    jvp,
    vjp,
    interactions,
    num_threads,
    set_num_threads,
)
from .brute import brute_accel  # noqa: F401
from .multipoles import abs_moments, multipoles, terms  # noqa: F401
from .stepping import choose_step, kick_drift, step_bounds, step_stats  # noqa: F401
