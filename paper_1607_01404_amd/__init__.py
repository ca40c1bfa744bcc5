"""MI355X (gfx950) two-stage hybrid partial SVD (PHSVDS) -- Python binding.

The binding only marshals arguments: device tensors (PyTorch is used for
device memory and streams) are passed as raw pointers to the C ABI declared in
include/svds.h, and every step of the solver runs in the library's HIP
kernels.  If the built library is missing, importing the entry points raises.
"""
from ._lib import (  # noqa: F401
    LARGEST,
    SMALLEST,
    FP64,
    MIXED,
    PC_NONE,
    PC_JACOBI,
    PC_LEARNED,
    PC_BLOCKJACOBI,
    METHOD_HYBRID,
    METHOD_NORMAL,
    METHOD_AUGMENTED,
    STAGE2_GDK,
    STAGE2_JD,
    condest,
    blockjacobi_apply,
    LPC_NPARAMS,
    SvdsError,
    Opts,
    Stats,
    library_path,
    load_library,
    opts_init,
    error_string,
    Matrix,
    solve,
    solve_batched,
    svds,
    small_eig,
    small_svd,
    lpc_init,
    lpc_features,
    lpc_forward,
    lpc_backward,
    lpc_loss,
    lpc_apply,
    lpc_adam,
    lpc_train,
    collect_residuals,
    stream_release,
)
