"""MI355X-native shifted-Laplace rational-filter eigensolver (ParaSLRF hot path).

The compute path is the HIP shared library ``libslrf.so`` (built by
``paper_2510_17334_amd.build``); this package only marshals arguments to its
C ABI.  PyTorch provides all device memory (inputs, outputs and each handle's
workspace) and the stream.  There is no CPU
fallback: every entry point raises if the library is missing.
"""

from .slrf import (  # noqa: F401
    SLRF_PREC_FP64,
    SLRF_PREC_MIXED,
    SLRF_PC_NONE,
    SLRF_PC_JACOBI,
    SLRF_PC_AMG,
    SLRF_AMG_HOST,
    SLRF_AMG_DEVICE,
    SlrfError,
    Handle,
    EigFn,
    default_options,
    lib,
    library_path,
    host_projected_eig,
    KERNEL_CLASSES,
    slrf_filter_batch,
    slrf_solve_batch,
    workspace_size,
)
