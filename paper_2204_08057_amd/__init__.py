"""MI355X (gfx950) solver for the posterior mean of the CMB source-separation model.

Python binding of libsylv (C ABI declared in include/sylv.h).  Argument marshalling only: every
numerical step runs in the library's HIP kernels; torch supplies device memory and the current
stream.  Importing works without a GPU; calling any solver function requires the built library
and a GPU, and raises otherwise (there is no CPU fallback).
"""
from .binding import (  # noqa: F401
    SYLV_BC_FACE,
    SYLV_BC_PERIODIC,
    SYLV_F32,
    SYLV_F64,
    SYLV_PC_BLOCK,
    SYLV_PC_JACOBI,
    SYLV_PC_NONE,
    SYLV_PREC_F64,
    SYLV_PREC_MIXED,
    SYLV_SCHED_ADAPTIVE,
    SYLV_SCHED_FIXED,
    SYLV_STOP_B,
    SYLV_STOP_R0,
    STATUS_NAMES,
    DeviceProblem,
    LanczosOptions,
    SepProblem,
    SolveOptions,
    SylvError,
    SylvSolve,
    apply,
    apply_launcher,
    autotune,
    declared_symbols,
    lanczos_solve,
    lanczos_workspace_bytes,
    lib,
    library_path,
    pcg_backward,
    pcg_solve,
    pcg_solve_noalloc,
    NOALLOC_SCRATCH_BYTES,
    po_perturb,
    precond,
    rhs,
    solve_launcher,
    stats_list,
    status_string,
    workspace_bytes,
)
