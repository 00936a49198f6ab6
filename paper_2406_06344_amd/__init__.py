"""MI355X (gfx950) implementation of the offline U/V build and the batched,
differentiated apply of the parametric Chebyshev / tensor-train kernel
low-rank method (Khan & Saibaba, arXiv 2406.06344).

The work runs in libttk.so (HIP kernels behind the C ABI of
include/tt_kernel.h); this package only marshals arguments.
"""
from .api import HMatrix, TTBatch, TTKernel, eval_dense, eval_entries, kernel_apply, make_params  # noqa: F401
