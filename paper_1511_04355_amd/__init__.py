"""afsbem: MI355X-native per-frequency Laplace-domain elastodynamic BEM solve.

Thin Python binding over the C ABI of ``libafsbem.so`` (see ``include/afsbem.h``).
Every step of the solve runs in the library's HIP kernels; PyTorch only owns
device memory and provides the stream.  Importing this package does not load
the library; the first call does, and fails loudly if it has not been built.
"""
from ._lib import (  # noqa: F401
    AfsbemError,
    FMT_C128,
    FMT_SPLIT,
    PREC_FP64,
    PREC_MIXED,
    WARM_NONE,
    WARM_PREV,
    WARM_USER,
    WARM_LEARNED,
    WARM_MODEL,
    WARM_EXTRAP,
    WARM_USER_AUG,
    Problem,
    SolveOptions,
    solve_batched,
    hmat_partition_info,
    plan_info,
    autotune_set,
    autotune_report,
    lib,
    lib_path,
    version,
    fsm_grid,
    fsm_invert,
    vf_fit,
    vf_residues,
    vf_eval,
    vf_eval_time,
    afs_params,
    time_synthesis,
    model_sample,
    fsm_invert_device,
    afs_run,
)
