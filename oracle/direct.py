"""Oracle (test infrastructure only): the exact solution x = A^{-1} b.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.

The linear system of the paper's Eq. (5) has the plain definition
x = A^{-1} b.  Small systems use a dense LU with partial pivoting
(LAPACK gesv through numpy.linalg.solve); larger ones a sparse LU (SuperLU
through scipy), both library routines used as single steps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def solve(A: sp.spmatrix, b: np.ndarray, transpose: bool = False) -> np.ndarray:
    M = A.T if transpose else A
    if A.shape[0] <= 6000:
        return np.linalg.solve(M.toarray(), b)
    return spl.splu(sp.csc_matrix(M)).solve(b)
