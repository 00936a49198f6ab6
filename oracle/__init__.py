"""Plain FP64 CPU oracle for the parametric Chebyshev / tensor-train kernel
low-rank method (PTTK) of Khan & Saibaba, "Parametric kernel low-rank
approximations using tensor train decomposition" (arXiv 2406.06344).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke entry
point and the benchmark's CPU-baseline leg may import it.  The product path
(the C-ABI library and its Python binding) never calls into it, and it shares
no code, tables or constants with that path.

Everything here is written for obviousness, not speed: NumPy/SciPy in float64,
one function per step of the paper, each citing the passage it follows.

Modules
-------
rng      counter-based generator (splitmix64) that keys every random draw the
         cross algorithm makes; the GPU library implements the same published
         generator independently.
basis    Chebyshev nodes, affine map, Lagrange basis as a Chebyshev sum
         (Section 2.4) and its theta-derivative.
kernels  the kernel table (Table 1) plus two test kernels, and the entry
         function f_kappa on the Chebyshev grid (Section 1, "Our approach";
         Section 2.4, "Multivariate approximation").
tt       TT format helpers: unfoldings, full reconstruction, TT-SVD,
         TT-Round (Algorithm 1).
cross    TT greedy-cross: index initialisation (Algorithm 7), the update
         cross step (Algorithm 5), the outline (Algorithm 6) and the
         interpolation formula (Appendix A).
pttk     offline Phase 3 (Algorithm 2), the rounding/gauge step used by the
         GPU path, the online stage (Algorithm 3), derivatives, the apply and
         its backward pass, and PTTK-Global-1 (Algorithm 4).
dense    dense kernel matrices and the error metrics of Section 4.
"""
