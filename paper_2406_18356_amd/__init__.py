"""MI355X (gfx950) minor-cycle solver of the two-step radio-interferometric
reconstruction (Wang, Prunet, Mignot & Ferrari, "Multi-Step Reconstruction of
Radio-Interferometric Images").

The compute path is the HIP library ``libmsr.so`` built from ``csrc/`` (see
``include/msr.h`` for the C ABI).  This package is a thin ctypes binding over
it: PyTorch supplies device memory and streams, every arithmetic step runs in
the library's kernels.  Importing the binding fails loudly when the library
is missing.
"""
from .binding import (  # noqa: F401
    MsrError,
    Config,
    SolveOptions,
    Result,
    Solver,
    Batch,
    UNet,
    unet_layers,
    unet_init_params,
    lib,
    library_path,
    abi_version,
    workspace_bytes,
    SYMBOLS,
)
