"""FP64 CPU oracle for the two-stage hybrid partial SVD (PHSVDS).

TEST INFRASTRUCTURE ONLY.  Only the test suite, smoke() in __graft_entry__.py
and the CPU-baseline leg of the benchmark may import or run anything in this
package.  The library (the HIP path and its Python binding)
never imports it, and it imports nothing from the library.

Parity unpinned: iteration and matrix-vector counts (they depend on the
readings of the unspecified GD+k details); everything the solver returns is
pinned by the CPU tests (LAPACK SVD on small matrices, prescribed singular
values, closed-form sparse families, the residual and orthonormality
invariants, the spectrum of the augmented matrix and the stage-1 bracket).
"""
from .phsvds import (  # noqa: F401
    EPS,
    counter_uniform,
    Operators,
    estimate_norm,
    ortho_block,
    jacobi_diag,
    block_jacobi,
    exact_inverse,
    svds,
    svd_residuals,
    condest,
    minres,
    sqmr,
)
