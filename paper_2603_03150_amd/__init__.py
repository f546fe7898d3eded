"""MI355X (gfx950) restarted PDHG for standard-form LPs, behind the C ABI of
include/mipdhg.h.  The Python layer only marshals device pointers."""
from ._lib import (  # noqa: F401
    OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, IN_PROGRESS, MipdhgError, load,
)
from .solver import (  # noqa: F401
    BatchSolution, DeviceBatch, autotune, DeviceLP, Solution, batch_workspace_bytes, default_options, make_options,
    center_reclamp, center_start, solve, solve_batched, workspace_bytes, state_bytes, export_state, import_state,
    read_probe, IpmSolution, ipm_options, ipm_solve, ipm_warm, autotune_batched,
)
from .unrolled import PDHGUnrolled, UnrolledMap  # noqa: F401
