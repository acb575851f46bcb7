"""CPU oracle: plain, slow, FP64 reference implementation of the solver.

This package is test infrastructure.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path (the HIP
library and its Python binding) never does and shares no code with it.

Modules: nd (nested dissection), spand (factor / apply / apply^T),
krylov (classical and s-step GMRES), direct (A^{-1} b), adjoint
(reference gradients).  Each function cites the passage it follows.
"""
