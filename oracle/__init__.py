"""CPU oracle for the shift-and-invert low-rank method (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library and its
Python binding never import, call or link it, and it shares no code with them.

Each function cites the passage of the paper it follows.  Everything the paper
leaves open (the inner solver's schedule, the sampler, the gap estimate, the
stopping rule) is implemented with one fixed reading; see the module
docstrings.
"""
from .philox import philox4x32_10, gaussian_block, key_of, stream_word  # noqa: F401
from .sampling import column_sq_norms, build_table, step_indices, mulhi64, draw  # noqa: F401
from .linalg import cholqr, cholqr2, eigh_desc, jacobi_svd, sin_theta, sign_fix  # noqa: F401
from .lowrank import (  # noqa: F401
    Options, Schedule, Result, LowRankError, solve, decode, apply_A, estimate_phase,
    solver_constants, svrg_step, svrg_solve, tune_shift, si_iterate, final_rr,
    LR_OK, LR_EINVAL, LR_ENOMEM, LR_ENOGAP, LR_ENOCONV, LR_ESHIFT, LR_ENOTSPD,
)
from .adaptive import (  # noqa: F401
    solve_adaptive, large_detect, delta_detect, estimate_deflated, power_deflated, si_deflated,
)
from .lowrank import deflate  # noqa: F401
from .lowrank import inner_schedule, inner_solve  # noqa: F401
from .accel import accel_constants, acc_svrg_solve  # noqa: F401
