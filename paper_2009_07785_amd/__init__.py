"""MI355X (gfx950) domain propagation: synchronous activity-based bound
tightening of lhs <= Ax <= rhs in hand-written HIP kernels behind a C ABI
(include/prop.h).  Importing the package loads libprop.so and fails if it
has not been built."""
from .binding import (  # noqa: F401
    CONVERGED,
    INFEASIBLE,
    MAX_ROUNDS,
    STATUS_NAMES,
    Problem,
    PropError,
    RunResult,
    Server,
    autotune,
)
