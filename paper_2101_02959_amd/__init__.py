"""MI355X-native Newton-Krylov BDDC / FETI-DP deluxe solver for the
segregated implicit Bidomain time step.

The compute path is libbidomain.so (hand-written HIP for gfx950) behind the C
ABI in include/bidomain.h; ``paper_2101_02959_amd.bidomain`` marshals
arguments to it with ctypes.  Importing this package does not load the
library; ``bidomain.lib()`` does, and raises if it has not been built.
"""
from .bidomain import (BDM_FETI_F, BDM_FETI_PRECOND, BDM_FETI_RECOVER, BDM_FETI_RHS,  # noqa: F401
                       BDM_GUESS_CNN, BDM_GUESS_EXTRAP, BDM_GUESS_PREV, BDM_KERNEL_JACOBIAN,
                       BDM_KERNEL_POTRF_INTERIOR, BDM_KERNEL_SYRK_UPDATE, BDM_KERNEL_TRSV_DIRICHLET,
                       BDM_KERNEL_TRSV_DIRICHLET_T, BDM_PREC_FP64, BDM_PREC_MIXED, BDM_SCHED_GRID,
                       BDM_SCHED_QUEUE, BDM_SOLVER_BDDC, BDM_SOLVER_FETIDP, BidomainError, Solver, lib,
                       BDM_SCALING_DELUXE, BDM_SCALING_RHO, BDM_PRIMAL_VE, BDM_PRIMAL_V, BDM_PRIMAL_VEF,
                       bdm_residual_noalloc)
